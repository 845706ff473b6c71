// swe_run_static: start and step a state without any device allocation by the caller or the
// library.  The step partials and arrival counters that swe_state_init and swe_run keep in the
// caller's workspace live here in one library-owned device array per GPU instead.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>
#include <string>

#include "swe_internal.h"

// Partials and counters of one state's steps, for meshes whose workspace (swe_workspace_bytes)
// fits SWE_STATIC_WORK_BYTES.  Every GPU the library runs on holds its own copy until the
// process ends; every call on that GPU shares it.
static __device__ __align__(256) unsigned char scratch[SWE_STATIC_WORK_BYTES];

namespace swe {
namespace {

// Device address of each GPU's copy, looked up once per device (host code never uses the
// array's own name as an address).
void *g_scratch_ptr[64] = {};
std::mutex g_scratch_mu;

int32_t sfail(int32_t code, const std::string &msg)
{
    set_error(msg);
    return code;
}

// Arrival counters must read zero, and the step's slots +inf (the bound's bits), 0 and 0, when
// a state's steps begin: n_count counters, n_slot slots.
__global__ void clear_counters_kernel(Partials part, int64_t n_count, int64_t n_slot)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n_count) part.count[i] = 0u;
    if (i < n_slot) {
        reinterpret_cast<unsigned long long *>(part.dt)[i] = kInfBits;
        part.clamps[i] = 0;
        part.flags[i] = 0;
    }
}

}  // namespace
}  // namespace swe

using namespace swe;

extern "C" int32_t swe_run_static(const swe_mesh *mesh, const swe_dev_mesh *dm,
                                  const swe_params *p, swe_state *s, int32_t init, double t0,
                                  double t_end, int64_t n_steps, const double *dt_seq,
                                  swe_run_stats *out, void *stream)
{
    if (!mesh || !dm || !p || !s) return sfail(SWE_EINVAL, "swe_run_static: null argument");
    if (n_steps < 0) return sfail(SWE_EINVAL, "swe_run_static: n_steps < 0");
    if (dt_seq && n_steps < 1) return sfail(SWE_EINVAL, "swe_run_static: dt_seq needs n_steps >= 1");
    if (init && (!isfinite(t0) || !isfinite(t_end)))
        return sfail(SWE_EINVAL, "swe_run_static: t0 and t_end must be finite");
    const int64_t nb = n_tiles_of(mesh->info.n_cells, mesh->info.tile_cells);
    const int64_t need = workspace_bytes_for_tiles(nb);
    if (need > static_cast<int64_t>(SWE_STATIC_WORK_BYTES))
        return sfail(SWE_EINVAL, "swe_run_static: the mesh needs " + std::to_string(need) +
                                     " bytes of step partials, beyond the static " +
                                     std::to_string(SWE_STATIC_WORK_BYTES) +
                                     " (use swe_run with a workspace)");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return sfail(SWE_EDEVICE, "swe_run_static: no current device below index 64");
    void *work = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return sfail(SWE_EDEVICE, std::string("swe_run_static: hipGetSymbolAddress: ") +
                                              hipGetErrorString(e));
            g_scratch_ptr[dev] = ptr;
        }
        work = g_scratch_ptr[dev];
    }
    // the same calls as swe_state_init and swe_run, on a copy of the state whose workspace is
    // this device's array; swe_run's graphs are not used (their instantiation may allocate)
    swe_state st = *s;
    st.work = work;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const Partials part = partials_for(work, nb);
    const int64_t n_count = n_groups(nb) + 1, n_slot = n_slots(nb);
    const int64_t n_clear = n_count > n_slot ? n_count : n_slot;
    clear_counters_kernel<<<dim3(static_cast<unsigned>((n_clear + 255) / 256)), 256, 0, hs>>>(
        part, n_count, n_slot);
    if (hipGetLastError() != hipSuccess)
        return sfail(SWE_EDEVICE, "swe_run_static: counter clear failed to launch");
    if (init) {
        if (int32_t rc = swe_state_init(mesh, dm, p, &st, t0, t_end, stream)) return rc;
    }
    if (int32_t rc = run_steps(mesh, dm, p, &st, n_steps, dt_seq, false, stream)) return rc;
    s->cur = st.cur;
    if (!out) return SWE_OK;
    return swe_read_stats(s, out, stream);
}
