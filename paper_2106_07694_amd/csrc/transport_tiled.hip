// transport_tiled.hip -- launchers of the tiled RK3 stage kernels
// (transport_tiled.h) and the kernels with a constant settling speed.
#include "transport_tiled.h"

namespace lbw {

TileShape resolve_tile_shape(int dim, const lbw_launch &l) {
    TileShape s;
    if (dim == 3) {
        s.tx = (l.tile_x == 64 || l.tile_x == 128) ? l.tile_x : 32;
        s.ty = 256 / s.tx;
        if ((s.tx == 32 && l.tile_rows == 16) || (s.tx == 64 && l.tile_rows == 8)) s.ty = l.tile_rows;
    } else {
        s.tx = (l.tile_x == 64 || l.tile_x == 128 || l.tile_x == 512) ? l.tile_x : 256;
        s.ty = 1;
    }
    s.chunk = l.tile_y > 0 ? l.tile_y : (dim == 3 ? 64 : 32);
    return s;
}

int64_t transport_tiles(int dim, const RunDev &r, const lbw_launch &l) {
    const TileShape s = resolve_tile_shape(dim, l);
    const TileGeom g = dim == 3 ? make_geom<3>(r, s.chunk, s.tx, s.ty) : make_geom<2>(r, s.chunk, s.tx, s.ty);
    return (int64_t)g.gx * g.gy * g.gz;
}

hipError_t launch_transport_tiled(int dim, int precision, const RunDev &r, const lbw_launch &l,
                                  hipStream_t st) {
    if (r.vs_s != 0.0) return launch_transport_tiled_vs(dim, precision, r, l, st, nullptr);
    return tiled_any<false>(dim, precision, r, l, st, nullptr);
}

hipError_t launch_one_stage(int dim, int precision, const RunDev &r, const lbw_launch &l,
                            int stage, hipStream_t st) {
    if (r.vs_s != 0.0) return hipErrorInvalidValue;   // built for a constant settling speed
    if (precision == LBW_FP32_SHIFTED)
        return dim == 2 ? one_stage_d<float, 2>(r, l, stage, st) : one_stage_d<float, 3>(r, l, stage, st);
    return dim == 2 ? one_stage_d<double, 2>(r, l, stage, st) : one_stage_d<double, 3>(r, l, stage, st);
}

hipError_t launch_transport_batched(int dim, int precision, const BatchArgs &b, const lbw_launch &l,
                                    hipStream_t st) {
    const RunDev &r = b.host_runs[0];
    bool any_var = false, any_const = false;
    for (int i = 0; i < b.nbatch; ++i) (b.host_runs[i].vs_s != 0.0 ? any_var : any_const) = true;
    if (!any_var) return tiled_any<false>(dim, precision, r, l, st, &b);
    if (!any_const) return launch_transport_tiled_vs(dim, precision, r, l, st, &b);
    // both settling forms: each stage runs once per form, each kernel over
    // its own entries, so every run takes the kernels it takes alone
    BatchArgs x = b;
    for (int k = 1; k <= 3; ++k) {
        hipError_t e = hipSuccess;
        x.stage = k;
        x.form = 0;
        if (e == hipSuccess) e = tiled_any<false>(dim, precision, r, l, st, &x);
        x.form = 1;
        if (e == hipSuccess) e = launch_transport_tiled_vs(dim, precision, r, l, st, &x);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lbw
