// Launchers of libswe that pick the kernels' FP64 arithmetic: swe::exact (correctly rounded
// division and square root, bitwise the host's IEEE operations) or swe::fast (hardware-seeded
// Newton forms, within an ulp).  FP32 is the same in both; the mode-free launchers use exact's.
#include <hip/hip_runtime.h>

#include "swe_internal.h"

namespace swe {

int launch_init(int dtype, const swe_dev_mesh &dm, const StepConfig &cfg, const swe_state &s,
                double t0, double t_end, void *stream, const BatchLaunch *batch)
{
    return cfg.fast ? fast::launch_init(dtype, dm, cfg, s, t0, t_end, stream, batch)
                    : exact::launch_init(dtype, dm, cfg, s, t0, t_end, stream, batch);
}

int launch_step(int dtype, const swe_dev_mesh &dm, const StepConfig &cfg, const swe_state &s,
                int cur, const double *dt_seq, int64_t n_seq, void *stream, const TileLayout *tl,
                const BatchLaunch *batch, int remap, double *const *ustar,
                const double *dt_direct)
{
    return cfg.fast ? fast::launch_step(dtype, dm, cfg, s, cur, dt_seq, n_seq, stream, tl, batch,
                                        remap, ustar, dt_direct)
                    : exact::launch_step(dtype, dm, cfg, s, cur, dt_seq, n_seq, stream, tl, batch,
                                         remap, ustar, dt_direct);
}

size_t tile_lds_bytes_for(int dtype, const TileLayout &tl)
{
    return exact::tile_lds_bytes_for(dtype, tl);
}

int prepare_tile_kernels(size_t max_lds)
{
    if (int e = exact::prepare_tile_kernels(max_lds)) return e;
    return fast::prepare_tile_kernels(max_lds);
}

int launch_run_begin(const swe_state &s, const double *dt_seq, void *stream)
{
    return exact::launch_run_begin(s, dt_seq, stream);
}

int launch_halo(int dtype, bool pack, int64_t n, const int32_t *idx, const void *buf_in,
                void *buf_out, const void *h, const void *hu, const void *hv, void *ho, void *huo,
                void *hvo, void *stream)
{
    return exact::launch_halo(dtype, pack, n, idx, buf_in, buf_out, h, hu, hv, ho, huo, hvo,
                              stream);
}

int launch_shard_combine(void *const *ctrls, int n, void *stream)
{
    return exact::launch_shard_combine(ctrls, n, stream);
}

int launch_flux_eval(int dtype, int64_t n, double g, double h_dry, const void *hl,
                     const void *hul, const void *hvl, const void *zl, const void *hr,
                     const void *hur, const void *hvr, const void *zr, const void *nx,
                     const void *ny, void *f, void *p, void *stream)
{
    return exact::launch_flux_eval(dtype, n, g, h_dry, hl, hul, hvl, zl, hr, hur, hvr, zr, nx,
                                   ny, f, p, stream);
}

int launch_flux_eval(int dtype, bool fast_math, int64_t n, double g, double h_dry,
                     const void *hl, const void *hul, const void *hvl, const void *zl,
                     const void *hr, const void *hur, const void *hvr, const void *zr,
                     const void *nx, const void *ny, void *f, void *p, void *stream)
{
    return fast_math ? fast::launch_flux_eval(dtype, n, g, h_dry, hl, hul, hvl, zl, hr, hur, hvr,
                                              zr, nx, ny, f, p, stream)
                     : exact::launch_flux_eval(dtype, n, g, h_dry, hl, hul, hvl, zl, hr, hur,
                                               hvr, zr, nx, ny, f, p, stream);
}

}  // namespace swe
