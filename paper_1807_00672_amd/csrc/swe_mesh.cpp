// Host-side mesh builder of libswe: orientation, interface matching, boundary codes, Morton
// renumbering of cells and first-touch renumbering of nodes.
//
// The paper's domain is a set of triangles (section 2.2, eq. 3) and its flux loop runs over
// interfaces (section 2.3).  The step kernels instead gather per cell, so the builder turns
// the triangle list into per-cell neighbour lists in an order that keeps neighbours close in
// memory.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "swe_internal.h"

namespace {

using swe::kEdgeA;
using swe::kEdgeKa;
using swe::kEdgeKb;
using swe::n_tiles_of;
using swe::valid_tile;

struct Fail {
    int32_t code;
    std::string msg;
};

inline uint32_t spread_bits(uint32_t v)  // 16 bits -> even bit positions of 32
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Position of the cell (x, y) of a 65536 x 65536 grid along a Hilbert curve: at each scale,
// take the quadrant, add the cells of the quadrants the curve visits before it, and rotate or
// reflect the coordinates into the quadrant's own orientation.
inline uint32_t hilbert_key(uint32_t x, uint32_t y)
{
    const uint32_t n = 1u << 16;
    uint32_t d = 0;
    for (uint32_t s = n >> 1; s > 0; s >>= 1) {
        const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = n - 1 - x;
                y = n - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

// Stable LSD radix sort of (key, index) by a 32-bit key, two 16-bit passes.
void radix_sort_by_key(std::vector<uint32_t> &key, std::vector<int32_t> &idx)
{
    const size_t n = key.size();
    std::vector<uint32_t> k2(n);
    std::vector<int32_t> i2(n);
    for (int pass = 0; pass < 2; ++pass) {
        const int sh = 16 * pass;
        std::vector<size_t> cnt(65537, 0);
        for (size_t i = 0; i < n; ++i) ++cnt[((key[i] >> sh) & 0xffffu) + 1];
        for (size_t b = 1; b <= 65536; ++b) cnt[b] += cnt[b - 1];
        for (size_t i = 0; i < n; ++i) {
            const size_t d = cnt[(key[i] >> sh) & 0xffffu]++;
            k2[d] = key[i];
            i2[d] = idx[i];
        }
        key.swap(k2);
        idx.swap(i2);
    }
}

// Tiles of tile_cells consecutive mesh-order cells.  Per tile: the halo (cells outside it that
// share an edge with it, ascending) and the edge list: every interface between two tile
// cells once (owned by the lower local index), every interface to a halo cell or the
// boundary once (owned by the tile cell).  Interior and halo entries come first, boundary
// entries last, so that the waves evaluating them branch alike.  slot[k*T + i] points cell
// i's local edge k at its entry, bit 15 marking the side b of an interior interface.
void build_tiles(swe_mesh &m)
{
    const int64_t T = m.info.n_cells;
    const int64_t TB = m.info.tile_cells;
    if (!valid_tile(TB)) throw Fail{SWE_EINVAL, "tile size must be 64, 128, 256 or 512"};
    const int64_t nt = n_tiles_of(T, TB);
    m.halo_off.assign(nt + 1, 0);
    m.edge_off.assign(nt + 1, 0);
    m.halo.clear();
    m.edges.clear();
    m.slot.assign(3 * T, 0);
    int32_t max_halo = 0, max_edges = 0;
    std::vector<int32_t> hl;
    std::vector<uint32_t> inner, bnd;
    std::vector<int32_t> inner_cell, bnd_cell;  // (local cell * 4 + k) of each entry
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t s0 = t * TB, s1 = std::min<int64_t>(T, s0 + TB);
        hl.clear();
        for (int64_t i = s0; i < s1; ++i)
            for (int k = 0; k < 3; ++k) {
                const int32_t j = m.nbr[k * T + i];
                if (j >= 0 && (j < s0 || j >= s1)) hl.push_back(j);
            }
        std::sort(hl.begin(), hl.end());
        hl.erase(std::unique(hl.begin(), hl.end()), hl.end());
        if (static_cast<int64_t>(hl.size()) > 32767 - TB)
            throw Fail{SWE_EMESH, "tile halo too large"};
        inner.clear(); bnd.clear(); inner_cell.clear(); bnd_cell.clear();
        for (int64_t i = s0; i < s1; ++i) {
            const uint32_t a = static_cast<uint32_t>(i - s0);
            for (int k = 0; k < 3; ++k) {
                const int32_t j = m.nbr[k * T + i];
                int32_t b;
                if (j >= s0 && j < s1) {
                    if (j < i) continue;  // owned by the lower local index
                    b = static_cast<int32_t>(j - s0);
                } else if (j >= 0) {
                    b = static_cast<int32_t>(TB) + static_cast<int32_t>(
                                       std::lower_bound(hl.begin(), hl.end(), j) - hl.begin());
                } else {
                    b = j;
                }
                const uint32_t w = a | (static_cast<uint32_t>(k) << kEdgeKa) |
                                   (static_cast<uint32_t>(static_cast<uint16_t>(static_cast<int16_t>(b))) << 16);
                if (b >= 0) {
                    inner.push_back(w);
                    inner_cell.push_back(static_cast<int32_t>(a) * 4 + k);
                } else {
                    bnd.push_back(w);
                    bnd_cell.push_back(static_cast<int32_t>(a) * 4 + k);
                }
            }
        }
        const int32_t n_inner = static_cast<int32_t>(inner.size());
        for (int32_t e = 0; e < n_inner + static_cast<int32_t>(bnd.size()); ++e) {
            const uint32_t w = e < n_inner ? inner[e] : bnd[e - n_inner];
            const int32_t ak = e < n_inner ? inner_cell[e] : bnd_cell[e - n_inner];
            const int64_t i = s0 + ak / 4;
            const int k = ak % 4;
            m.slot[k * T + i] = static_cast<uint16_t>(e);
            const int32_t b = static_cast<int16_t>(w >> 16);
            uint32_t wk = w;
            if (b >= 0 && b < TB) {  // side b of an interior interface
                const int64_t jb = s0 + b;
                int kb = -1;
                for (int q = 0; q < 3; ++q)
                    if (m.nbr[q * T + jb] == i) kb = q;
                if (kb < 0) throw Fail{SWE_EMESH, "neighbour relation is not mutual"};
                m.slot[kb * T + jb] = static_cast<uint16_t>(e | 0x8000);
                wk |= static_cast<uint32_t>(kb) << kEdgeKb;   // b's local edge, for the tile's slots
            }
            m.edges.push_back(wk);
        }
        m.halo.insert(m.halo.end(), hl.begin(), hl.end());
        m.halo_off[t + 1] = static_cast<int32_t>(m.halo.size());
        m.edge_off[t + 1] = static_cast<int32_t>(m.edges.size());
        max_halo = std::max(max_halo, static_cast<int32_t>(hl.size()));
        max_edges = std::max(max_edges, n_inner + static_cast<int32_t>(bnd.size()));
    }
    if (m.edges.size() > static_cast<size_t>(INT32_MAX) || m.halo.size() > static_cast<size_t>(INT32_MAX))
        throw Fail{SWE_EINVAL, "mesh too large for int32 tile offsets"};
    // each entry's edge vector, node k+1 minus node k of its owning cell (eq. 3's outward
    // normal is (dy, -dx) / l), so that the step reads it instead of two node lookups
    m.edge_vec.resize(2 * m.edges.size());
    for (int64_t t = 0; t < nt; ++t)
        for (int32_t e = m.edge_off[t]; e < m.edge_off[t + 1]; ++e) {
            const uint32_t w = m.edges[e];
            const int64_t ca = t * TB + static_cast<int64_t>(w & kEdgeA);
            const int k = static_cast<int>((w >> kEdgeKa) & 3u);
            const int32_t n0 = m.c2n[k * T + ca], n1 = m.c2n[((k + 1) % 3) * T + ca];
            m.edge_vec[2 * static_cast<size_t>(e)] = m.xy[2 * static_cast<size_t>(n1)] - m.xy[2 * static_cast<size_t>(n0)];
            m.edge_vec[2 * static_cast<size_t>(e) + 1] =
                m.xy[2 * static_cast<size_t>(n1) + 1] - m.xy[2 * static_cast<size_t>(n0) + 1];
        }
    // each tile's nodes in first-use order and, per entry, the tile-local ids of the nodes
    // whose difference is its edge vector: the FP64 tiled step stages a tile's nodes (about
    // 0.7 per cell) once instead of reading an edge vector per entry (about 1.7 per cell);
    // kept only where every tile's ids fit in 8 bits and its nodes number at most its cells
    // (one per work-item)
    const int32_t node_cap = static_cast<int32_t>(std::min<int64_t>(256, TB));
    std::vector<int32_t> local(static_cast<size_t>(m.info.n_nodes), -1);
    std::vector<int32_t> used;
    int32_t max_nodes = 0;
    m.tile_node_off.assign(nt + 1, 0);
    m.tile_nodes.clear();
    m.edge_nodes.assign(m.edges.size(), 0);
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t s0 = t * TB, s1 = std::min<int64_t>(T, s0 + TB);
        used.clear();
        for (int64_t i = s0; i < s1; ++i)
            for (int k = 0; k < 3; ++k) {
                const int32_t v = m.c2n[k * T + i];
                if (local[v] < 0) {
                    local[v] = static_cast<int32_t>(used.size());
                    used.push_back(v);
                }
            }
        max_nodes = std::max(max_nodes, static_cast<int32_t>(used.size()));
        if (max_nodes <= node_cap) {
            for (int32_t e = m.edge_off[t]; e < m.edge_off[t + 1]; ++e) {
                const uint32_t w = m.edges[e];
                const int64_t ca = s0 + static_cast<int64_t>(w & kEdgeA);
                const int k = static_cast<int>((w >> kEdgeKa) & 3u);
                const int32_t n0 = local[m.c2n[k * T + ca]], n1 = local[m.c2n[((k + 1) % 3) * T + ca]];
                m.edge_nodes[e] = static_cast<uint16_t>(n0 | (n1 << 8));
            }
            for (int32_t v : used) {
                m.tile_nodes.push_back(m.xy[2 * static_cast<size_t>(v)]);
                m.tile_nodes.push_back(m.xy[2 * static_cast<size_t>(v) + 1]);
            }
            m.tile_node_off[t + 1] = static_cast<int32_t>(m.tile_nodes.size() / 2);
        }
        for (int32_t v : used) local[v] = -1;
    }
    if (max_nodes > node_cap || m.tile_nodes.size() / 2 > static_cast<size_t>(INT32_MAX)) {
        m.tile_node_off.clear();
        m.tile_nodes.clear();
        m.edge_nodes.clear();
    }
    m.info.n_tile_nodes = static_cast<int64_t>(m.tile_nodes.size() / 2);
    m.info.max_tile_nodes = max_nodes;
    m.info.n_tiles = nt;
    m.info.n_halo = static_cast<int64_t>(m.halo.size());
    m.info.n_tile_edges = static_cast<int64_t>(m.edges.size());
    m.info.max_halo = max_halo;
    m.info.max_tile_edges = max_edges;
    m.tiles.n_tiles = nt;
    m.tiles.max_halo = max_halo;
    m.tiles.max_edges = max_edges;
    m.tiles.max_nodes = m.tile_nodes.empty() ? 0 : max_nodes;
    m.tiles.tile = static_cast<int32_t>(TB);
}

void build(swe_mesh &m, const double *xy, int64_t nv, const int32_t *tri, int64_t nt,
           const int32_t *tags, uint32_t flags)
{
    if (!xy || !tri) throw Fail{SWE_EINVAL, "null xy or tri"};
    if (nv < 3 || nt < 1) throw Fail{SWE_EINVAL, "need at least 3 nodes and 1 triangle"};
    if (nv > INT32_MAX / 2 || nt > INT32_MAX / 3)
        throw Fail{SWE_EINVAL, "mesh too large for int32 indices"};
    if (flags & ~(SWE_MORTON | SWE_HILBERT | SWE_TILE_64 | SWE_TILE_128 | SWE_TILE_512))
        throw Fail{SWE_EINVAL, "unknown flags"};
    const uint32_t tf = flags & (SWE_TILE_64 | SWE_TILE_128 | SWE_TILE_512);
    if (tf & (tf - 1)) throw Fail{SWE_EINVAL, "more than one tile size flag"};
    const int32_t tile = tf == SWE_TILE_64 ? 64 : tf == SWE_TILE_128 ? 128 : tf == SWE_TILE_512 ? 512 : SWE_TILE;
    if ((flags & SWE_MORTON) && (flags & SWE_HILBERT))
        throw Fail{SWE_EINVAL, "SWE_MORTON and SWE_HILBERT exclude each other"};
    for (int64_t j = 0; j < 2 * nv; ++j)
        if (!isfinite(xy[j])) throw Fail{SWE_EINVAL, "non-finite node coordinate"};

    const int64_t T = nt;
    // 1. counter-clockwise triangles, local order kept; clockwise ones become (v0, v2, v1)
    std::vector<int32_t> cn(3 * T), ct(3 * T, 0);
    int32_t max_tag = 0;
    for (int64_t c = 0; c < T; ++c) {
        int32_t v0 = tri[3 * c], v1 = tri[3 * c + 1], v2 = tri[3 * c + 2];
        if (v0 < 0 || v1 < 0 || v2 < 0 || v0 >= nv || v1 >= nv || v2 >= nv)
            throw Fail{SWE_EMESH, "triangle " + std::to_string(c) + " has a node out of range"};
        if (v0 == v1 || v1 == v2 || v0 == v2)
            throw Fail{SWE_EMESH, "triangle " + std::to_string(c) + " repeats a node"};
        const double e0x = xy[2 * v1] - xy[2 * v0], e0y = xy[2 * v1 + 1] - xy[2 * v0 + 1];
        const double e1x = xy[2 * v2] - xy[2 * v1], e1y = xy[2 * v2 + 1] - xy[2 * v1 + 1];
        const double cr = e0x * e1y - e0y * e1x;
        if (!(cr != 0.0)) throw Fail{SWE_EMESH, "triangle " + std::to_string(c) + " has zero area"};
        int32_t t0 = 0, t1 = 0, t2 = 0;
        if (tags) {
            t0 = tags[3 * c]; t1 = tags[3 * c + 1]; t2 = tags[3 * c + 2];
            if (t0 < 0 || t1 < 0 || t2 < 0 || t0 > SWE_MAX_INFLOW || t1 > SWE_MAX_INFLOW ||
                t2 > SWE_MAX_INFLOW)
                throw Fail{SWE_EINVAL, "edge tag out of range [0, SWE_MAX_INFLOW]"};
        }
        if (cr < 0.0) {
            std::swap(v1, v2);
            std::swap(t0, t2);
        }
        cn[3 * c] = v0; cn[3 * c + 1] = v1; cn[3 * c + 2] = v2;
        ct[3 * c] = t0; ct[3 * c + 1] = t1; ct[3 * c + 2] = t2;
    }

    // 2. match half-edges: bucket by their smaller node (counting sort), pair within buckets
    std::vector<int64_t> start(nv + 1, 0);
    for (int64_t h = 0; h < 3 * T; ++h) {
        const int32_t a = cn[h], b = cn[(h / 3) * 3 + (h % 3 + 1) % 3];
        ++start[std::min(a, b) + 1];
    }
    for (int64_t j = 0; j < nv; ++j) start[j + 1] += start[j];
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    std::vector<int32_t> bucket(3 * T);
    for (int64_t h = 0; h < 3 * T; ++h) {
        const int32_t a = cn[h], b = cn[(h / 3) * 3 + (h % 3 + 1) % 3];
        bucket[fill[std::min(a, b)]++] = static_cast<int32_t>(h);
    }
    std::vector<int32_t> nb_old(3 * T, SWE_WALL);
    int64_t ne = 0, nbnd = 0, ninflow = 0;
    for (int64_t lo = 0; lo < nv; ++lo) {
        const int64_t s0 = start[lo], s1 = start[lo + 1];
        for (int64_t x = s0; x < s1; ++x) {
            const int32_t h = bucket[x];
            if (h < 0) continue;  // already paired
            const int32_t c = h / 3, k = h % 3;
            const int32_t a = cn[h], b = cn[3 * c + (k + 1) % 3];
            const int32_t hi = std::max(a, b);
            int32_t mate = -1;
            for (int64_t y = x + 1; y < s1; ++y) {
                const int32_t g = bucket[y];
                if (g < 0) continue;
                const int32_t cg = g / 3, kg = g % 3;
                const int32_t ag = cn[g], bg = cn[3 * cg + (kg + 1) % 3];
                if (std::max(ag, bg) != hi) continue;
                if (mate >= 0)
                    throw Fail{SWE_EMESH, "edge (" + std::to_string(a) + "," + std::to_string(b) +
                                              ") is shared by more than two triangles"};
                if (ag == a)
                    throw Fail{SWE_EMESH, "triangles " + std::to_string(c) + " and " +
                                              std::to_string(cg) + " overlap along an edge"};
                mate = static_cast<int32_t>(y);
            }
            ++ne;
            if (mate >= 0) {
                const int32_t g = bucket[mate];
                nb_old[h] = g / 3;
                nb_old[g] = c;
                bucket[mate] = -1;
            } else {
                ++nbnd;
                const int32_t tg = ct[h];
                nb_old[h] = tg > 0 ? -1 - tg : SWE_WALL;
                if (tg > 0) {
                    ++ninflow;
                    max_tag = std::max(max_tag, tg);
                }
            }
            bucket[x] = -1;
        }
    }

    // 3. geometry summary and centroids
    swe_mesh_info &inf = m.info;
    memset(&inf, 0, sizeof(inf));
    inf.n_cells = T;
    inf.n_owned = T;
    inf.n_nodes = nv;
    inf.n_edges = ne;
    inf.n_boundary_edges = nbnd;
    inf.n_inflow_edges = ninflow;
    inf.n_inflow_segments = max_tag;
    inf.flags = flags;
    inf.tile_cells = tile;
    inf.min_area = INFINITY;
    inf.min_inradius = INFINITY;
    inf.bbox[0] = inf.bbox[1] = INFINITY;
    inf.bbox[2] = inf.bbox[3] = -INFINITY;
    for (int64_t j = 0; j < nv; ++j) {
        inf.bbox[0] = std::min(inf.bbox[0], xy[2 * j]);
        inf.bbox[1] = std::min(inf.bbox[1], xy[2 * j + 1]);
        inf.bbox[2] = std::max(inf.bbox[2], xy[2 * j]);
        inf.bbox[3] = std::max(inf.bbox[3], xy[2 * j + 1]);
    }
    std::vector<uint32_t> key(T);
    const double sx = inf.bbox[2] > inf.bbox[0] ? 65535.0 / (inf.bbox[2] - inf.bbox[0]) : 0.0;
    const double sy = inf.bbox[3] > inf.bbox[1] ? 65535.0 / (inf.bbox[3] - inf.bbox[1]) : 0.0;
    for (int64_t c = 0; c < T; ++c) {
        const int32_t *v = &cn[3 * c];
        double per = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double dx = xy[2 * v[(k + 1) % 3]] - xy[2 * v[k]];
            const double dy = xy[2 * v[(k + 1) % 3] + 1] - xy[2 * v[k] + 1];
            per += sqrt(dx * dx + dy * dy);
        }
        const double e0x = xy[2 * v[1]] - xy[2 * v[0]], e0y = xy[2 * v[1] + 1] - xy[2 * v[0] + 1];
        const double e1x = xy[2 * v[2]] - xy[2 * v[1]], e1y = xy[2 * v[2] + 1] - xy[2 * v[1] + 1];
        const double a = 0.5 * (e0x * e1y - e0y * e1x);
        inf.min_area = std::min(inf.min_area, a);
        inf.max_area = std::max(inf.max_area, a);
        inf.total_area += a;
        inf.min_inradius = std::min(inf.min_inradius, 2.0 * a / per);
        const double cx = (xy[2 * v[0]] + xy[2 * v[1]] + xy[2 * v[2]]) / 3.0;
        const double cy = (xy[2 * v[0] + 1] + xy[2 * v[1] + 1] + xy[2 * v[2] + 1]) / 3.0;
        const uint32_t qx = static_cast<uint32_t>(std::min(65535.0, std::max(0.0, (cx - inf.bbox[0]) * sx)));
        const uint32_t qy = static_cast<uint32_t>(std::min(65535.0, std::max(0.0, (cy - inf.bbox[1]) * sy)));
        key[c] = (flags & SWE_HILBERT) ? hilbert_key(qx, qy)
                                       : spread_bits(qx) | (spread_bits(qy) << 1);
    }

    // 4. cell order: Morton or Hilbert key, ties by input index (stable sort of increasing
    // indices); else the input order
    m.perm.resize(T);
    for (int64_t c = 0; c < T; ++c) m.perm[c] = static_cast<int32_t>(c);
    if (flags & (SWE_MORTON | SWE_HILBERT)) radix_sort_by_key(key, m.perm);
    std::vector<int32_t> inv(T);
    for (int64_t i = 0; i < T; ++i) inv[m.perm[i]] = static_cast<int32_t>(i);

    // 5. nodes in order of first use by the renumbered cells; unused nodes last
    std::vector<int32_t> node_new(nv, -1);
    m.node_perm.clear();
    m.node_perm.reserve(nv);
    for (int64_t i = 0; i < T; ++i)
        for (int k = 0; k < 3; ++k) {
            const int32_t v = cn[3 * m.perm[i] + k];
            if (node_new[v] < 0) {
                node_new[v] = static_cast<int32_t>(m.node_perm.size());
                m.node_perm.push_back(v);
            }
        }
    for (int64_t j = 0; j < nv; ++j)
        if (node_new[j] < 0) {
            node_new[j] = static_cast<int32_t>(m.node_perm.size());
            m.node_perm.push_back(static_cast<int32_t>(j));
        }

    // 6. structure-of-arrays neighbour and node lists in mesh order
    m.nbr.resize(3 * T);
    m.c2n.resize(3 * T);
    for (int64_t i = 0; i < T; ++i) {
        const int32_t c = m.perm[i];
        for (int k = 0; k < 3; ++k) {
            const int32_t o = nb_old[3 * c + k];
            m.nbr[k * T + i] = o >= 0 ? inv[o] : o;
            m.c2n[k * T + i] = node_new[cn[3 * c + k]];
        }
    }
    m.xy.resize(2 * nv);
    for (int64_t j = 0; j < nv; ++j) {
        m.xy[2 * j] = xy[2 * m.node_perm[j]];
        m.xy[2 * j + 1] = xy[2 * m.node_perm[j] + 1];
    }
    // 7. area A = cross(e0, e1) / 2 and inradius r = 2A / P of every cell (eq. 4's A_i and the
    // CFL bound's length), with the edge vectors of its local edges in their order; IEEE
    // square root and division, evaluated in this order
    m.cell_geo.resize(2 * T);
    for (int64_t i = 0; i < T; ++i) {
        double ex[3], ey[3];
        for (int k = 0; k < 3; ++k) {
            const int32_t n0 = m.c2n[k * T + i], n1 = m.c2n[((k + 1) % 3) * T + i];
            ex[k] = m.xy[2 * static_cast<size_t>(n1)] - m.xy[2 * static_cast<size_t>(n0)];
            ey[k] = m.xy[2 * static_cast<size_t>(n1) + 1] - m.xy[2 * static_cast<size_t>(n0) + 1];
        }
        double l[3];
        for (int k = 0; k < 3; ++k) l[k] = sqrt(ex[k] * ex[k] + ey[k] * ey[k]);
        const double area = 0.5 * (ex[0] * ey[1] - ey[0] * ex[1]);
        m.cell_geo[i] = area;
        m.cell_geo[T + i] = (2.0 * area) / (l[0] + l[1] + l[2]);
    }
    build_tiles(m);
}

// Shard [c0, c1) of `full` and its halo as a mesh of its own (swe_mesh_create_shard).
void build_shard(swe_mesh &m, const swe_mesh &full, int64_t c0, int64_t c1)
{
    const int64_t T = full.info.n_cells;
    if (c0 < 0 || c1 <= c0 || c1 > T) throw Fail{SWE_EINVAL, "bad cell range"};
    std::vector<int32_t> cells;
    cells.reserve(static_cast<size_t>(c1 - c0));
    for (int64_t i = c0; i < c1; ++i) cells.push_back(static_cast<int32_t>(i));
    std::vector<int32_t> halo;
    for (int64_t i = c0; i < c1; ++i)
        for (int k = 0; k < 3; ++k) {
            const int32_t j = full.nbr[k * T + i];
            if (j >= 0 && (j < c0 || j >= c1)) halo.push_back(j);
        }
    std::sort(halo.begin(), halo.end());
    halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
    cells.insert(cells.end(), halo.begin(), halo.end());
    const int64_t n = static_cast<int64_t>(cells.size());
    // nodes the shard uses, numbered in the full mesh's order
    std::vector<int32_t> node_of(static_cast<size_t>(full.info.n_nodes), -1);
    std::vector<int32_t> nodes;
    for (int32_t c : cells)
        for (int k = 0; k < 3; ++k) {
            const int32_t v = full.c2n[k * T + c];
            if (node_of[v] < 0) {
                node_of[v] = 0;
                nodes.push_back(v);
            }
        }
    std::sort(nodes.begin(), nodes.end());
    for (size_t q = 0; q < nodes.size(); ++q) node_of[nodes[q]] = static_cast<int32_t>(q);
    std::vector<double> xy(2 * nodes.size());
    for (size_t q = 0; q < nodes.size(); ++q) {
        xy[2 * q] = full.xy[2 * static_cast<size_t>(nodes[q])];
        xy[2 * q + 1] = full.xy[2 * static_cast<size_t>(nodes[q]) + 1];
    }
    // triangles in the full mesh's (counter-clockwise) node order; inflow tags kept
    std::vector<int32_t> tri(3 * n), tag(3 * n, 0);
    for (int64_t q = 0; q < n; ++q)
        for (int k = 0; k < 3; ++k) {
            const int32_t c = cells[q];
            tri[3 * q + k] = node_of[full.c2n[k * T + c]];
            const int32_t code = full.nbr[k * T + c];
            if (code < SWE_WALL) tag[3 * q + k] = -1 - code;
        }
    // the full mesh's tile size; no renumbering
    build(m, xy.data(), static_cast<int64_t>(nodes.size()), tri.data(), n, tag.data(),
          full.info.flags & (SWE_TILE_64 | SWE_TILE_128 | SWE_TILE_512));
    m.info.n_owned = c1 - c0;
    m.global = std::move(cells);
}

}  // namespace

extern "C" {

int32_t swe_mesh_create_shard(const swe_mesh *full, int64_t c0, int64_t c1, swe_mesh **out)
{
    if (!out || !full) {
        swe::set_error("swe_mesh_create_shard: null argument");
        return SWE_EINVAL;
    }
    *out = nullptr;
    swe_mesh *m = nullptr;
    try {
        m = new swe_mesh();
        build_shard(*m, *full, c0, c1);
    } catch (const Fail &f) {
        delete m;
        swe::set_error("swe_mesh_create_shard: " + f.msg);
        return f.code;
    } catch (const std::bad_alloc &) {
        delete m;
        swe::set_error("swe_mesh_create_shard: out of host memory");
        return SWE_EINVAL;
    } catch (...) {
        delete m;
        swe::set_error("swe_mesh_create_shard: unexpected failure");
        return SWE_EINVAL;
    }
    *out = m;
    return SWE_OK;
}

int32_t swe_mesh_create(const double *xy, int64_t nv, const int32_t *tri, int64_t nt,
                        const int32_t *edge_tag, uint32_t flags, swe_mesh **out)
{
    if (!out) {
        swe::set_error("swe_mesh_create: null out");
        return SWE_EINVAL;
    }
    *out = nullptr;
    swe_mesh *m = nullptr;
    try {
        m = new swe_mesh();
        build(*m, xy, nv, tri, nt, edge_tag, flags);
    } catch (const Fail &f) {
        delete m;
        swe::set_error("swe_mesh_create: " + f.msg);
        return f.code;
    } catch (const std::bad_alloc &) {
        delete m;
        swe::set_error("swe_mesh_create: out of host memory");
        return SWE_EINVAL;
    } catch (...) {
        delete m;
        swe::set_error("swe_mesh_create: unexpected failure");
        return SWE_EINVAL;
    }
    *out = m;
    return SWE_OK;
}

int32_t swe_mesh_info_get(const swe_mesh *mesh, swe_mesh_info *out)
{
    if (!mesh || !out) {
        swe::set_error("swe_mesh_info_get: null argument");
        return SWE_EINVAL;
    }
    *out = mesh->info;
    return SWE_OK;
}

int32_t swe_mesh_export(const swe_mesh *mesh, int32_t which, void *dst, int64_t dst_bytes)
{
    if (!mesh || !dst) {
        swe::set_error("swe_mesh_export: null argument");
        return SWE_EINVAL;
    }
    const void *src = nullptr;
    int64_t bytes = 0;
    switch (which) {
    case SWE_ARR_PERM: src = mesh->perm.data(); bytes = 4 * (int64_t)mesh->perm.size(); break;
    case SWE_ARR_NBR: src = mesh->nbr.data(); bytes = 4 * (int64_t)mesh->nbr.size(); break;
    case SWE_ARR_C2N: src = mesh->c2n.data(); bytes = 4 * (int64_t)mesh->c2n.size(); break;
    case SWE_ARR_XY: src = mesh->xy.data(); bytes = 8 * (int64_t)mesh->xy.size(); break;
    case SWE_ARR_NODE_PERM:
        src = mesh->node_perm.data(); bytes = 4 * (int64_t)mesh->node_perm.size(); break;
    case SWE_ARR_HALO_OFF:
        src = mesh->halo_off.data(); bytes = 4 * (int64_t)mesh->halo_off.size(); break;
    case SWE_ARR_HALO: src = mesh->halo.data(); bytes = 4 * (int64_t)mesh->halo.size(); break;
    case SWE_ARR_EDGE_OFF:
        src = mesh->edge_off.data(); bytes = 4 * (int64_t)mesh->edge_off.size(); break;
    case SWE_ARR_EDGES: src = mesh->edges.data(); bytes = 4 * (int64_t)mesh->edges.size(); break;
    case SWE_ARR_SLOT: src = mesh->slot.data(); bytes = 2 * (int64_t)mesh->slot.size(); break;
    case SWE_ARR_EDGE_VEC: src = mesh->edge_vec.data(); bytes = 8 * (int64_t)mesh->edge_vec.size(); break;
    case SWE_ARR_CELL_GEO: src = mesh->cell_geo.data(); bytes = 8 * (int64_t)mesh->cell_geo.size(); break;
    case SWE_ARR_EDGE_VEC32: return swe::export_as_float(mesh->edge_vec, dst, dst_bytes, "swe_mesh_export");
    case SWE_ARR_CELL_GEO32: return swe::export_as_float(mesh->cell_geo, dst, dst_bytes, "swe_mesh_export");
    case SWE_ARR_TILE_NODE_OFF:
        src = mesh->tile_node_off.data(); bytes = 4 * (int64_t)mesh->tile_node_off.size(); break;
    case SWE_ARR_TILE_NODES:
        src = mesh->tile_nodes.data(); bytes = 8 * (int64_t)mesh->tile_nodes.size(); break;
    case SWE_ARR_EDGE_NODES:
        src = mesh->edge_nodes.data(); bytes = 2 * (int64_t)mesh->edge_nodes.size(); break;
    case SWE_ARR_GLOBAL:
        bytes = 4 * mesh->info.n_cells;
        if (!mesh->global.empty()) {
            src = mesh->global.data();
            break;
        }
        if (dst_bytes < bytes) break;   // reported below
        for (int64_t i = 0; i < mesh->info.n_cells; ++i)   // not a shard: the identity
            static_cast<int32_t *>(dst)[i] = static_cast<int32_t>(i);
        return SWE_OK;
    default:
        swe::set_error("swe_mesh_export: unknown array " + std::to_string(which));
        return SWE_EINVAL;
    }
    if (dst_bytes < bytes) {
        swe::set_error("swe_mesh_export: destination holds " + std::to_string(dst_bytes) +
                       " bytes, array needs " + std::to_string(bytes));
        return SWE_EINVAL;
    }
    if (bytes > 0) memcpy(dst, src, static_cast<size_t>(bytes));
    return SWE_OK;
}

void swe_mesh_destroy(swe_mesh *mesh) { delete mesh; }

}  // extern "C"
