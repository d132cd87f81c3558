// api.cpp -- the C ABI declared in include/lbw.h: argument validation, the
// per-step launch sequence and the canonical export/import of fields.  The
// library never allocates device memory and synchronises only in lbw_reduce.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <mutex>
#include <vector>

#include "lbw_internal.h"

struct lbw_handle {
    int nbatch = 0;
    int q = 9, dim = 2, precision = LBW_FP64, fluid_mode = LBW_FLUID_LBM, scheme = LBW_WENO5;
    int has_s = 0;
    hipStream_t stream = nullptr;
    std::vector<lbw_config> cfg;
    std::vector<lbw_buffers> buf;
    std::vector<lbw::RunDev> run;
    int64_t steps = 0;
    bool odd = false;  // next collide-stream kernel is the odd one of the pair
    lbw_launch launch{256, 0, 0, 0, 0, 0, 0};
    // timing: spans (phase, start, end) drawn from a pool of events
    bool timing = false;
    struct Span {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Span> spans;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    int64_t timed_steps = 0;
    bool sflip = false;              // S currently lives in s_tmp
    int num_cu = 256;
    // batched mode (nbatch > 1): tables in run 0's scratch.  The transport
    // walks one entry per run and size class (`views`).
    lbw::RunDev *d_runs = nullptr, *d_views = nullptr;
    int *d_blk = nullptr, *d_tiles = nullptr;
    std::vector<int> blk_start, tile_start;
    std::vector<lbw::RunDev> views;
    int grid_lbm = 0, grid_tr = 0;
    // graph replay
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_odd = false, graph_sflip = false;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(LBW_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t elem_size(int precision) { return precision == LBW_FP32_SHIFTED ? 4 : 8; }

struct ScratchLayout {
    size_t out, runs, blk, views, tiles, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int classes_of(const lbw_config &c) { return c.n_classes > 1 ? c.n_classes : 1; }

// nviews: runs times their size classes (the transport's work items)
ScratchLayout scratch_layout(int nbatch, int nviews) {
    ScratchLayout L;
    L.out = sizeof(double) * (size_t)nbatch * lbw::kReduceBlocks;
    L.runs = align256(L.out + sizeof(double) * nbatch);
    if (nbatch > 1) {
        L.blk = align256(L.runs + sizeof(lbw::RunDev) * nbatch);
        L.views = align256(L.blk + sizeof(int) * (nbatch + 1));
        L.tiles = align256(L.views + sizeof(lbw::RunDev) * nviews);
        L.total = align256(L.tiles + sizeof(int) * (nviews + 1));
    } else {
        L.blk = L.views = L.tiles = L.total = L.runs;
    }
    return L;
}

int count_views(const lbw_config *cfgs, int nbatch) {
    int n = 0;
    for (int b = 0; b < nbatch; ++b) n += classes_of(cfgs[b]);
    return n;
}

// The run as the kernels must see it now (S and its work buffer swap roles
// after every step).
lbw::RunDev current(const lbw_handle *h, int b) {
    lbw::RunDev r = h->run[b];
    if (h->sflip) std::swap(r.s, r.s2);
    return r;
}

// Size class i of a run as the transport kernels see it: its C field and
// RK stage buffers, its deposit counters, its settling speed and
// diffusivity; the S update rides with class 0 only.  Classes share nothing
// they write, so the batched transport runs them all in one launch.
lbw::RunDev class_view(const lbw_handle *h, const lbw::RunDev &r, int b, int i) {
    if (r.ncls <= 1) return r;
    const lbw_config &c = h->cfg[b];
    lbw::RunDev v = r;
    const size_t off = (size_t)i * r.N * (h->precision == LBW_FP32_SHIFTED ? 4 : 8);
    v.c = (char *)r.c + off;
    v.c1 = (char *)r.c1 + off;
    v.c2 = (char *)r.c2 + off;
    v.dep = r.dep + (size_t)i * r.ncol;
    v.vs = c.vs_class[i];
    v.kappa_c = c.kappa_class[i];
    if (i > 0) v.has_s = 0;
    return v;
}

void release_graph(lbw_handle *h) {
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
}

// Work lists of the batched kernels for the current launch shape, copied
// into the scratch tables (ordered on the handle's stream).
int upload_tables(lbw_handle *h) {
    if (h->nbatch < 2) return LBW_OK;
    const int block = h->launch.lbm_block;
    h->blk_start.assign(h->nbatch + 1, 0);
    h->views.clear();
    for (int b = 0; b < h->nbatch; ++b) {
        const int64_t nb = (h->run[b].N + block - 1) / block;
        if ((int64_t)h->blk_start[b] + nb > 0x7fffffff)
            return fail(LBW_ERR_INVAL, "batched work list too large");
        h->blk_start[b + 1] = h->blk_start[b] + (int)nb;
        for (int i = 0; i < h->run[b].ncls; ++i) h->views.push_back(class_view(h, h->run[b], b, i));
    }
    const int nviews = (int)h->views.size();
    h->tile_start.assign(nviews + 1, 0);
    for (int v = 0; v < nviews; ++v) {
        const int64_t nt = lbw::transport_tiles(h->dim, h->views[v], h->launch);
        if ((int64_t)h->tile_start[v] + nt > 0x7fffffff)
            return fail(LBW_ERR_INVAL, "batched work list too large");
        h->tile_start[v + 1] = h->tile_start[v] + (int)nt;
    }
    const int per_cu_lbm = 2048 / block;
    h->grid_lbm = std::min(h->blk_start[h->nbatch], h->num_cu * per_cu_lbm);
    h->grid_tr = std::min(h->tile_start[nviews], h->num_cu * 8);
    hipError_t e = hipMemcpyAsync(h->d_runs, h->run.data(), sizeof(lbw::RunDev) * h->nbatch,
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->d_blk, h->blk_start.data(), sizeof(int) * (h->nbatch + 1),
                           hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->d_views, h->views.data(), sizeof(lbw::RunDev) * nviews,
                           hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->d_tiles, h->tile_start.data(), sizeof(int) * (nviews + 1),
                           hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // host tables may change later
    return e == hipSuccess ? LBW_OK : hip_fail(e, "upload of the batched work lists");
}

int validate(const lbw_config &c, const lbw_buffers &b, int idx) {
    if (c.lattice != LBW_D2Q9 && c.lattice != LBW_D3Q19)
        return fail(LBW_ERR_INVAL, "run %d: lattice must be LBW_D2Q9 or LBW_D3Q19", idx);
    if (c.precision != LBW_FP64 && c.precision != LBW_FP32_SHIFTED && c.precision != LBW_FP64_SHIFTED)
        return fail(LBW_ERR_INVAL, "run %d: unknown precision %d", idx, c.precision);
    if (c.n_classes < 0 || c.n_classes > LBW_MAX_CLASSES)
        return fail(LBW_ERR_INVAL, "run %d: n_classes must lie in [0, %d]", idx, LBW_MAX_CLASSES);
    if (c.nx < 1 || c.ny < 1 || c.nz < 1) return fail(LBW_ERR_INVAL, "run %d: grid sizes must be >= 1", idx);
    const int dim = c.lattice == LBW_D2Q9 ? 2 : 3;
    if (dim == 2 && c.nz != 1) return fail(LBW_ERR_INVAL, "run %d: D2Q9 needs nz == 1", idx);
    const int nv = dim == 2 ? c.ny : c.nz;
    if (nv < 6) return fail(LBW_ERR_INVAL, "run %d: vertical extent %d < 6 (one WENO5 stencil)", idx, nv);
    const int64_t N = (int64_t)c.nx * c.ny * c.nz;
    const int64_t lateral = dim == 2 ? (int64_t)c.nx : (int64_t)c.nx * c.ny;
    if (lateral * 8 >= ((int64_t)1 << 32))
        return fail(LBW_ERR_INVAL, "run %d: a horizontal plane must hold fewer than 2^29 cells", idx);
    // the per-node kernels launch one work-item per cell, and a dispatch
    // holds fewer than 2^32 work-items
    if (N > ((int64_t)1 << 32) - 1024)
        return fail(LBW_ERR_INVAL, "run %d: grid too large (%lld cells; at most 2^32 - 1024)", idx,
                    (long long)N);
    if (c.fluid_mode != LBW_FLUID_LBM && c.fluid_mode != LBW_FLUID_FROZEN)
        return fail(LBW_ERR_INVAL, "run %d: unknown fluid mode", idx);
    if (c.scheme_c != LBW_WENO5 && c.scheme_c != LBW_WENO3 && c.scheme_c != LBW_UPWIND1)
        return fail(LBW_ERR_INVAL, "run %d: unknown scheme", idx);
    if (c.fluid_mode == LBW_FLUID_LBM && !(c.tau > 0.5))
        return fail(LBW_ERR_INVAL, "run %d: tau = %g must exceed 1/2", idx, c.tau);
    if (!(c.vs >= 0.0) || c.vs > 1.0) return fail(LBW_ERR_INVAL, "run %d: vs must lie in [0, 1] (CFL)", idx);
    const double kmax = 1.0 / (2.0 * dim);
    if (!(c.kappa_c >= 0.0) || c.kappa_c > kmax)
        return fail(LBW_ERR_INVAL, "run %d: kappa_c must lie in [0, %g]", idx, kmax);
    if (c.n_classes > 1) {
        if (c.vs != 0.0 || c.kappa_c != 0.0)
            return fail(LBW_ERR_INVAL, "run %d: with size classes set vs_class and kappa_class "
                                       "(vs and kappa_c must be 0)", idx);
        for (int i = 0; i < c.n_classes; ++i) {
            if (!(c.vs_class[i] >= 0.0) || c.vs_class[i] > 1.0)
                return fail(LBW_ERR_INVAL, "run %d: vs_class[%d] must lie in [0, 1] (CFL)", idx, i);
            if (!(c.kappa_class[i] >= 0.0) || c.kappa_class[i] > kmax)
                return fail(LBW_ERR_INVAL, "run %d: kappa_class[%d] must lie in [0, %g]", idx, i, kmax);
        }
    }
    if (c.has_s && (!(c.kappa_s >= 0.0) || c.kappa_s > kmax))
        return fail(LBW_ERR_INVAL, "run %d: kappa_s must lie in [0, %g]", idx, kmax);
    if (!(c.weno_eps > 0.0)) return fail(LBW_ERR_INVAL, "run %d: weno_eps must be > 0", idx);
    for (int d = 0; d < 3; ++d) {
        if (!std::isfinite(c.body_force[d]) || !std::isfinite(c.u_top[d]) || std::fabs(c.u_top[d]) > 1.0)
            return fail(LBW_ERR_INVAL, "run %d: body force / lid velocity invalid", idx);
    }
    if (!std::isfinite(c.gp_c) || !std::isfinite(c.gp_s))
        return fail(LBW_ERR_INVAL, "run %d: buoyancy coefficients must be finite", idx);
    if (!std::isfinite(c.vs_s) || !std::isfinite(c.phi_c))
        return fail(LBW_ERR_INVAL, "run %d: vs_s and phi_c must be finite", idx);
    if ((c.vs_s != 0.0 || c.phi_c != 0.0) && !c.has_s)
        return fail(LBW_ERR_INVAL, "run %d: vs_s and phi_c act through S (has_s = 1)", idx);
    if (c.fluid_mode == LBW_FLUID_LBM && !b.f) return fail(LBW_ERR_INVAL, "run %d: f is NULL", idx);
    if (!b.c || !b.c_s1 || !b.c_s2) return fail(LBW_ERR_INVAL, "run %d: C buffers are NULL", idx);
    if (!b.u) return fail(LBW_ERR_INVAL, "run %d: u is NULL", idx);
    if (!b.deposit) return fail(LBW_ERR_INVAL, "run %d: deposit is NULL", idx);
    if (c.has_s && (!b.s || !b.s_tmp)) return fail(LBW_ERR_INVAL, "run %d: S buffers are NULL", idx);
    return LBW_OK;
}

lbw::RunDev make_run(const lbw_config &c, const lbw_buffers &b) {
    lbw::RunDev r{};
    r.f = b.f;
    r.c = b.c;
    r.c1 = b.c_s1;
    r.c2 = b.c_s2;
    r.s = b.s;
    r.s2 = b.s_tmp;
    r.u = b.u;
    r.rho = nullptr;
    r.dep = b.deposit;
    r.nx = c.nx;
    r.ny = c.ny;
    r.nz = c.nz;
    r.vper = c.vert_periodic ? 1 : 0;
    r.N = (int64_t)c.nx * c.ny * c.nz;
    r.ncol = c.lattice == LBW_D2Q9 ? c.nx : (int64_t)c.nx * c.ny;
    r.has_s = c.has_s ? 1 : 0;
    r.scheme = c.scheme_c;
    r.ncls = classes_of(c);
    r.tau = c.tau;
    r.omega = 1.0 / c.tau;
    r.guo = 1.0 - 0.5 / c.tau;
    for (int d = 0; d < 3; ++d) {
        r.body[d] = c.body_force[d];
        r.utop[d] = c.u_top[d];
    }
    r.vs = c.vs;
    r.kappa_c = c.kappa_c;
    r.gp_c = c.gp_c;
    r.kappa_s = c.kappa_s;
    r.gp_s = c.gp_s;
    r.eps = c.weno_eps;
    r.vs_s = c.vs_s;
    r.phi_c = c.phi_c;
    return r;
}

// A single run's tiled transport launches one block per tile and vertical
// chunk, and a dispatch holds fewer than 2^32 work-items: a huge run with
// short chunks and tiles that fit its lateral sizes badly could exceed that.
int check_tile_launch(const lbw_handle *h, const lbw_launch &l) {
    if (h->nbatch > 1 || l.variant == 1) return LBW_OK;   // persistent grid / one thread per node
    const lbw::TileShape s = lbw::resolve_tile_shape(h->dim, l);
    const int64_t items = lbw::transport_tiles(h->dim, h->run[0], l) * s.tx * s.ty;
    if (items >= ((int64_t)1 << 32))
        return fail(LBW_ERR_INVAL, "the transport launch would need %lld work-items (at most 2^32 - 1): "
                                   "choose a longer vertical chunk (tile_y)", (long long)items);
    return LBW_OK;
}

int check_run(const lbw_handle *h, int32_t run) {
    if (!h) return fail(LBW_ERR_INVAL, "NULL handle");
    if (run < 0 || run >= h->nbatch) return fail(LBW_ERR_INVAL, "run %d out of range [0, %d)", run, h->nbatch);
    return LBW_OK;
}

}  // namespace

extern "C" {

int lbw_version(void) { return LBW_ABI_VERSION; }

const char *lbw_last_error(void) { return g_err.c_str(); }

int lbw_scratch_bytes(const lbw_config *cfgs, int32_t nbatch, size_t *out_bytes) {
    if (!cfgs || nbatch < 1 || !out_bytes) return fail(LBW_ERR_INVAL, "bad arguments");
    *out_bytes = scratch_layout(nbatch, count_views(cfgs, nbatch)).total;
    return LBW_OK;
}

int lbw_create(const lbw_config *cfgs, const lbw_buffers *bufs, int32_t nbatch, void *stream,
               lbw_handle **out) {
    g_err.clear();
    if (!out) return fail(LBW_ERR_INVAL, "out is NULL");
    *out = nullptr;
    if (!cfgs || !bufs || nbatch < 1) return fail(LBW_ERR_INVAL, "need nbatch >= 1 configs and buffers");
    for (int b = 0; b < nbatch; ++b) {
        const int rc = validate(cfgs[b], bufs[b], b);
        if (rc) return rc;
        if (b > 0) {
            const lbw_config &a = cfgs[0], &c = cfgs[b];
            if (a.lattice != c.lattice || a.precision != c.precision || a.fluid_mode != c.fluid_mode ||
                a.scheme_c != c.scheme_c || a.has_s != c.has_s)
                return fail(LBW_ERR_INVAL, "run %d: batched runs must share lattice, precision, "
                                           "fluid mode, scheme and S option", b);
        }
    }
    lbw_handle *h = new (std::nothrow) lbw_handle;
    if (!h) return fail(LBW_ERR_INVAL, "out of host memory");
    h->nbatch = nbatch;
    h->q = cfgs[0].lattice;
    h->dim = h->q == LBW_D2Q9 ? 2 : 3;
    h->precision = cfgs[0].precision;
    h->fluid_mode = cfgs[0].fluid_mode;
    h->scheme = cfgs[0].scheme_c;
    h->has_s = cfgs[0].has_s;
    h->stream = (hipStream_t)stream;
    h->cfg.assign(cfgs, cfgs + nbatch);
    h->buf.assign(bufs, bufs + nbatch);
    for (int b = 0; b < nbatch; ++b) h->run.push_back(make_run(cfgs[b], bufs[b]));
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        h->num_cu = ncu;
    if (const int rc = check_tile_launch(h, h->launch)) {
        delete h;
        return rc;
    }
    if (nbatch > 1) {
        const ScratchLayout L = scratch_layout(nbatch, count_views(cfgs, nbatch));
        if (!bufs[0].scratch || bufs[0].scratch_bytes < L.total) {
            delete h;
            return fail(LBW_ERR_INVAL, "batched runs need %zu bytes of scratch in run 0", L.total);
        }
        char *base = (char *)bufs[0].scratch;
        h->d_runs = (lbw::RunDev *)(base + L.runs);
        h->d_blk = (int *)(base + L.blk);
        h->d_views = (lbw::RunDev *)(base + L.views);
        h->d_tiles = (int *)(base + L.tiles);
        const int rc = upload_tables(h);
        if (rc) {
            delete h;
            return rc;
        }
    }
    *out = h;
    return LBW_OK;
}

void lbw_destroy(lbw_handle *h) {
    if (!h) return;
    for (hipEvent_t ev : h->pool) (void)hipEventDestroy(ev);
    release_graph(h);
    delete h;
}

int lbw_set_launch(lbw_handle *h, const lbw_launch *l) {
    if (!h || !l) return fail(LBW_ERR_INVAL, "NULL argument");
    lbw_launch n = h->launch;
    if (l->lbm_block) {
        if (l->lbm_block < 64 || l->lbm_block > 1024 || l->lbm_block % 64)
            return fail(LBW_ERR_INVAL, "lbm_block must be a multiple of 64 in [64, 1024]");
        n.lbm_block = l->lbm_block;
    }
    if (l->tile_x) {
        const bool ok = h->dim == 3 ? (l->tile_x == 32 || l->tile_x == 64 || l->tile_x == 128)
                                    : (l->tile_x == 64 || l->tile_x == 128 || l->tile_x == 256 ||
                                       l->tile_x == 512);
        if (!ok) return fail(LBW_ERR_INVAL, "tile_x must be 32, 64 or 128 (3D) or 64, 128, 256 or 512 (2D)");
        n.tile_x = l->tile_x;
    }
    {
        const int tx = n.tile_x ? n.tile_x : (h->dim == 3 ? 32 : 256);
        const int tr = l->tile_rows;
        const bool ok = tr == 0 || (h->dim == 2 ? tr == 1
                                                : (tr == 256 / tx || (tx == 32 && tr == 16) ||
                                                   (tx == 64 && tr == 8)));
        if (!ok) return fail(LBW_ERR_INVAL, "tile_rows must be 0, 256 / tile_x, 16 (tile_x 32) or 8 (tile_x 64) in 3D, 0 or 1 in 2D");
        n.tile_rows = tr;
    }
    if (l->tile_y) {
        if (l->tile_y < 1 || l->tile_y > 4096) return fail(LBW_ERR_INVAL, "tile_y must lie in [1, 4096]");
        n.tile_y = l->tile_y;
    }
    if (l->variant < 0 || l->variant > 1) return fail(LBW_ERR_INVAL, "variant must be 0 or 1");
    n.variant = l->variant;
    if (l->reserved != 0) return fail(LBW_ERR_INVAL, "reserved must be 0");
    if (l->graph < 0 || l->graph > 1) return fail(LBW_ERR_INVAL, "graph must be 0 or 1");
    n.graph = l->graph;
    if (const int rc = check_tile_launch(h, n)) return rc;
    h->launch = n;
    release_graph(h);
    return upload_tables(h);
}

int lbw_get_launch(const lbw_handle *h, lbw_launch *l) {
    if (!h || !l) return fail(LBW_ERR_INVAL, "NULL argument");
    *l = h->launch;
    return LBW_OK;
}

int lbw_init_equilibrium(lbw_handle *h, int32_t run, const void *rho, const void *u) {
    int rc = check_run(h, run);
    if (rc) return rc;
    if (h->fluid_mode != LBW_FLUID_LBM) return fail(LBW_ERR_INVAL, "frozen fluid has no populations");
    hipError_t e = lbw::launch_equilibrium(h->q, h->precision, current(h, run), h->odd, rho, u, h->stream);
    return e == hipSuccess ? LBW_OK : hip_fail(e, "equilibrium");
}

namespace {
hipEvent_t pooled_event(lbw_handle *h) {
    if (h->pool_used < h->pool.size()) return h->pool[h->pool_used++];
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    h->pool.push_back(ev);
    ++h->pool_used;
    return ev;
}

// Open a timing span of `phase` on stream st (timing mode only); returns its
// index or -1.
int span_open(lbw_handle *h, int phase, hipStream_t st) {
    if (!h->timing) return -1;
    lbw_handle::Span sp{phase, pooled_event(h), pooled_event(h)};
    if (!sp.a || !sp.b || hipEventRecord(sp.a, st) != hipSuccess) return -2;
    h->spans.push_back(sp);
    return (int)h->spans.size() - 1;
}

int span_close(lbw_handle *h, int idx, hipStream_t st) {
    if (idx == -1) return LBW_OK;
    if (idx < 0) return fail(LBW_ERR_HIP, "timing event unavailable");
    hipError_t e = hipEventRecord(h->spans[idx].b, st);
    return e == hipSuccess ? LBW_OK : hip_fail(e, "event record");
}
}  // namespace

namespace {
// Enqueue one coupled step on the handle's stream and advance the host-side
// state (streaming parity, S buffer roles, step count).
int enqueue_step(lbw_handle *h) {
    int rc;
    int sp = span_open(h, LBW_PHASE_COLLIDE_STREAM, h->stream);
    if (h->fluid_mode == LBW_FLUID_LBM) {
        hipError_t e;
        if (h->nbatch > 1) {
            int64_t nodes = 0;
            for (const auto &rr : h->run) nodes += rr.N;
            e = lbw::launch_collide_stream_batched(h->q, h->precision, h->d_runs, h->d_blk, h->nbatch,
                                                   h->sflip ? 1 : 0, h->odd, h->launch.lbm_block,
                                                   h->grid_lbm, nodes, h->stream);
        }
        else
            e = lbw::launch_collide_stream(h->q, h->precision, current(h, 0), h->odd,
                                           h->launch.lbm_block, h->stream);
        if (e != hipSuccess) return hip_fail(e, "collide-stream launch");
    }
    if ((rc = span_close(h, sp, h->stream))) return rc;
    sp = span_open(h, LBW_PHASE_TRANSPORT, h->stream);
    if (h->nbatch > 1 && h->launch.variant == 0) {
        lbw::BatchArgs a;
        a.runs = h->d_views;
        a.tile_start = h->d_tiles;
        a.host_runs = h->views.data();
        a.nbatch = (int)h->views.size();
        a.chunk = lbw::resolve_tile_shape(h->dim, h->launch).chunk;
        a.sflip = h->sflip ? 1 : 0;
        a.grid = h->grid_tr;
        hipError_t e = lbw::launch_transport_batched(h->dim, h->precision, a, h->launch, h->stream);
        if (e != hipSuccess) return hip_fail(e, "batched transport launch");
    } else {
        for (int b = 0; b < h->nbatch; ++b) {
            const lbw::RunDev r = current(h, b);
            for (int i = 0; i < r.ncls; ++i) {
                hipError_t e = lbw::launch_transport(h->dim, h->precision, class_view(h, r, b, i),
                                                     h->launch, h->stream);
                if (e != hipSuccess) return hip_fail(e, "transport launch");
            }
        }
    }
    if ((rc = span_close(h, sp, h->stream))) return rc;
    if (h->timing) ++h->timed_steps;
    if (h->has_s) h->sflip = !h->sflip;
    if (h->fluid_mode == LBW_FLUID_LBM) h->odd = !h->odd;
    ++h->steps;
    return LBW_OK;
}

// Capture two steps from the current state into a graph (the state returns
// to where it was: two steps restore the parity and the S roles).
int build_graph(lbw_handle *h) {
    release_graph(h);
    const bool odd = h->odd, sflip = h->sflip;
    const int64_t steps = h->steps;
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "graph capture begin");
    int rc = enqueue_step(h);
    if (!rc) rc = enqueue_step(h);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->stream, &g);
    h->odd = odd;
    h->sflip = sflip;
    h->steps = steps;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "graph capture end");
    h->graph = g;
    e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        release_graph(h);
        return hip_fail(e, "graph instantiate");
    }
    h->graph_odd = odd;
    h->graph_sflip = sflip;
    return LBW_OK;
}
}  // namespace

int lbw_step(lbw_handle *h, int32_t nsteps) {
    if (!h) return fail(LBW_ERR_INVAL, "NULL handle");
    if (nsteps < 0) return fail(LBW_ERR_INVAL, "nsteps must be >= 0");
    int rc;
    if (h->launch.graph && !h->timing && nsteps >= 2) {
        if (!h->stream) return fail(LBW_ERR_UNSUPPORTED, "graph replay needs a non-null stream");
        if (!h->gexec || h->graph_odd != h->odd || h->graph_sflip != h->sflip)
            if ((rc = build_graph(h))) return rc;
        while (nsteps >= 2) {
            hipError_t e = hipGraphLaunch(h->gexec, h->stream);
            if (e != hipSuccess) return hip_fail(e, "graph launch");
            h->steps += 2;
            nsteps -= 2;
        }
    }
    for (int32_t s = 0; s < nsteps; ++s)
        if ((rc = enqueue_step(h))) return rc;
    return LBW_OK;
}

int lbw_adjoint_work_bytes(const lbw_handle *h, int32_t run, size_t *out_bytes) {
    int rc = check_run(h, run);
    if (rc) return rc;
    if (!out_bytes) return fail(LBW_ERR_INVAL, "out_bytes is NULL");
    *out_bytes = lbw::adjoint_work_bytes(h->dim, h->precision, h->run[run].N);
    return LBW_OK;
}

int lbw_adjoint_step(lbw_handle *h, int32_t run, const void *f_n, const void *c_n,
                     const void *u_n, const void *rho_n, const void *a1_n, const void *a2_n,
                     const void *fbar_next, const void *cbar_next, double dep_bar, void *fbar,
                     void *cbar, double *vs_bar_dev, void *work, size_t work_bytes) {
    int rc = check_run(h, run);
    if (rc) return rc;
    if (h->scheme != LBW_WENO5 || h->has_s || h->run[run].ncls > 1)
        return fail(LBW_ERR_UNSUPPORTED, "the adjoint covers WENO5 transport without S, one size class");
    const bool frozen = h->fluid_mode == LBW_FLUID_FROZEN;
    if (!c_n || !cbar_next || !cbar || !work) return fail(LBW_ERR_INVAL, "NULL required argument");
    if ((a1_n == nullptr) != (a2_n == nullptr))
        return fail(LBW_ERR_INVAL, "give both RK stages or neither");
    if (!frozen && (!fbar_next || !fbar))
        return fail(LBW_ERR_INVAL, "the population adjoints are required");
    if (!frozen && !f_n && !(u_n && rho_n))
        return fail(LBW_ERR_INVAL, "give the populations, or the velocity and the density");
    if (cbar == cbar_next || cbar == c_n || (!frozen && (fbar == fbar_next || fbar == f_n)))
        return fail(LBW_ERR_INVAL, "outputs must not alias inputs");
    if (!std::isfinite(dep_bar)) return fail(LBW_ERR_INVAL, "dep_bar must be finite");
    const size_t need = lbw::adjoint_work_bytes(h->dim, h->precision, h->run[run].N);
    if (work_bytes < need) return fail(LBW_ERR_INVAL, "work needs %zu bytes", need);
    hipError_t e = lbw::launch_adjoint(h->q, h->precision, h->run[run], frozen, f_n, c_n, u_n, rho_n,
                                       a1_n, a2_n, fbar_next, cbar_next, dep_bar, fbar, cbar, vs_bar_dev,
                                       work, h->launch, h->stream);
    return e == hipSuccess ? LBW_OK : hip_fail(e, "adjoint launch");
}

int lbw_timing_begin(lbw_handle *h) {
    if (!h) return fail(LBW_ERR_INVAL, "NULL handle");
    h->spans.clear();
    h->pool_used = 0;
    h->timed_steps = 0;
    h->timing = true;
    return LBW_OK;
}

int lbw_timing_end(lbw_handle *h, double *ms_out, int64_t *steps) {
    if (!h || !ms_out || !steps) return fail(LBW_ERR_INVAL, "NULL argument");
    h->timing = false;
    for (int p = 0; p < LBW_NPHASES; ++p) ms_out[p] = 0.0;
    *steps = h->timed_steps;
    int rc = LBW_OK;
    for (const auto &sp : h->spans) {
        hipError_t e = hipEventSynchronize(sp.b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, sp.a, sp.b);
        if (e != hipSuccess) {
            rc = hip_fail(e, "event elapsed");
            break;
        }
        ms_out[sp.phase] += ms;
    }
    h->spans.clear();
    h->pool_used = 0;
    return rc;
}

int lbw_steps_done(const lbw_handle *h, int64_t *out) {
    if (!h || !out) return fail(LBW_ERR_INVAL, "NULL argument");
    *out = h->steps;
    return LBW_OK;
}

int lbw_export(lbw_handle *h, int32_t run, int32_t field, void *dst) {
    int rc = check_run(h, run);
    if (rc) return rc;
    if (!dst) return fail(LBW_ERR_INVAL, "dst is NULL");
    const lbw::RunDev &r = h->run[run];
    const size_t es = elem_size(h->precision);
    hipError_t e = hipSuccess;
    switch (field) {
        case LBW_FIELD_F:
            if (h->fluid_mode != LBW_FLUID_LBM) return fail(LBW_ERR_INVAL, "frozen fluid has no populations");
            e = lbw::launch_export_f(h->q, h->precision, r, h->odd, dst, h->stream);
            break;
        case LBW_FIELD_C:
            e = hipMemcpyAsync(dst, r.c, r.ncls * r.N * es, hipMemcpyDeviceToDevice, h->stream);
            break;
        case LBW_FIELD_S:
            if (!h->has_s) return fail(LBW_ERR_INVAL, "run has no S");
            e = hipMemcpyAsync(dst, current(h, run).s, r.N * es, hipMemcpyDeviceToDevice, h->stream);
            break;
        case LBW_FIELD_U:
            e = hipMemcpyAsync(dst, r.u, (size_t)h->dim * r.N * es, hipMemcpyDeviceToDevice, h->stream);
            break;
        case LBW_FIELD_DEPOSIT:
            e = hipMemcpyAsync(dst, r.dep, r.ncls * r.ncol * sizeof(double), hipMemcpyDeviceToDevice,
                               h->stream);
            break;
        case LBW_FIELD_STAGE1:
            e = hipMemcpyAsync(dst, r.c1, r.ncls * r.N * es, hipMemcpyDeviceToDevice, h->stream);
            break;
        case LBW_FIELD_STAGE2:
            e = hipMemcpyAsync(dst, r.c2, r.ncls * r.N * es, hipMemcpyDeviceToDevice, h->stream);
            break;
        default: return fail(LBW_ERR_INVAL, "unknown field %d", field);
    }
    return e == hipSuccess ? LBW_OK : hip_fail(e, "export");
}

int lbw_rebind(lbw_handle *h, int32_t run, int32_t field, void *ptr) {
    int rc = check_run(h, run);
    if (rc) return rc;
    lbw::RunDev &r = h->run[run];
    const lbw_buffers &b = h->buf[run];
    switch (field) {
        case LBW_FIELD_U:
            if (h->fluid_mode != LBW_FLUID_LBM)
                return fail(LBW_ERR_INVAL, "a frozen velocity is an input: import it instead");
            r.u = ptr ? ptr : b.u;
            break;
        case LBW_FIELD_RHO:
            if (h->fluid_mode != LBW_FLUID_LBM) return fail(LBW_ERR_INVAL, "a frozen fluid has no density");
            r.rho = ptr;
            break;
        case LBW_FIELD_STAGE1: r.c1 = ptr ? ptr : b.c_s1; break;
        case LBW_FIELD_STAGE2: r.c2 = ptr ? ptr : b.c_s2; break;
        default: return fail(LBW_ERR_INVAL, "only U, RHO, STAGE1 and STAGE2 can be rebound (field %d)", field);
    }
    release_graph(h);
    return upload_tables(h);
}

int lbw_replay(lbw_handle *h, int32_t run, int32_t n, void *const *c_out, void *const *u_out,
               void *const *rho_out, void *const *a1_out, void *const *a2_out) {
    int rc = check_run(h, run);
    if (rc) return rc;
    if (n < 0) return fail(LBW_ERR_INVAL, "n must be >= 0");
    if (h->nbatch > 1) return fail(LBW_ERR_UNSUPPORTED, "lbw_replay drives a single run (a step advances every run of a batch)");
    const bool lbm = h->fluid_mode == LBW_FLUID_LBM;
    if (!c_out || !a1_out || !a2_out || (lbm && (!u_out || !rho_out)))
        return fail(LBW_ERR_INVAL, "NULL pointer array");
    for (int i = 0; i < n; ++i)
        if (!c_out[i] || !a1_out[i] || !a2_out[i] || (lbm && (!u_out[i] || !rho_out[i])))
            return fail(LBW_ERR_INVAL, "NULL buffer for replayed step %d", i);
    for (int i = 0; i < n && !rc; ++i) {
        rc = lbw_export(h, run, LBW_FIELD_C, c_out[i]);
        if (!rc && lbm) rc = lbw_rebind(h, run, LBW_FIELD_U, u_out[i]);
        if (!rc && lbm) rc = lbw_rebind(h, run, LBW_FIELD_RHO, rho_out[i]);
        if (!rc) rc = lbw_rebind(h, run, LBW_FIELD_STAGE1, a1_out[i]);
        if (!rc) rc = lbw_rebind(h, run, LBW_FIELD_STAGE2, a2_out[i]);
        if (!rc) rc = lbw_step(h, 1);
    }
    // bind the per-step outputs back to the handle's own buffers
    int rb = lbw_rebind(h, run, LBW_FIELD_STAGE1, nullptr);
    if (!rb) rb = lbw_rebind(h, run, LBW_FIELD_STAGE2, nullptr);
    if (!rb && lbm) rb = lbw_rebind(h, run, LBW_FIELD_U, nullptr);
    if (!rb && lbm) rb = lbw_rebind(h, run, LBW_FIELD_RHO, nullptr);
    return rc ? rc : rb;
}

int lbw_import(lbw_handle *h, int32_t run, int32_t field, const void *src) {
    int rc = check_run(h, run);
    if (rc) return rc;
    if (!src) return fail(LBW_ERR_INVAL, "src is NULL");
    const lbw::RunDev &r = h->run[run];
    const size_t es = elem_size(h->precision);
    hipError_t e = hipSuccess;
    switch (field) {
        case LBW_FIELD_F:
            if (h->fluid_mode != LBW_FLUID_LBM) return fail(LBW_ERR_INVAL, "frozen fluid has no populations");
            e = lbw::launch_import_f(h->q, h->precision, r, h->odd, src, h->stream);
            break;
        case LBW_FIELD_C:
            e = hipMemcpyAsync(r.c, src, r.ncls * r.N * es, hipMemcpyDeviceToDevice, h->stream);
            break;
        case LBW_FIELD_S:
            if (!h->has_s) return fail(LBW_ERR_INVAL, "run has no S");
            e = hipMemcpyAsync(current(h, run).s, src, r.N * es, hipMemcpyDeviceToDevice, h->stream);
            break;
        case LBW_FIELD_U:
            e = hipMemcpyAsync(r.u, src, (size_t)h->dim * r.N * es, hipMemcpyDeviceToDevice, h->stream);
            break;
        case LBW_FIELD_DEPOSIT:
            e = hipMemcpyAsync(r.dep, src, r.ncls * r.ncol * sizeof(double), hipMemcpyDeviceToDevice,
                               h->stream);
            break;
        default: return fail(LBW_ERR_INVAL, "unknown field %d", field);
    }
    return e == hipSuccess ? LBW_OK : hip_fail(e, "import");
}

// Device scratch of the no-allocation reduction (lbw_reduce_static): the
// per-block partial sums and the per-run results of up to kStaticRuns runs,
// laid out as in the caller's scratch (partials run after run, then the
// sums).  Each device holds its own copy; host code reaches it only through
// the address hipGetSymbolAddress returns for the device (the array's name
// is a host-side stand-in, not a device address).
constexpr int kStaticRuns = 128;
constexpr size_t kStaticDoubles = (size_t)kStaticRuns * lbw::kReduceBlocks + kStaticRuns;
static __device__ __align__(256) double scratch[kStaticDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// Address of `scratch` on the device the handle's stream runs on, looked up
// once per device with that device current.
int static_scratch(const lbw_handle *h, double **out) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int dev = cur;
    if (h->stream) {
        e = hipStreamGetDevice(h->stream, &dev);
        if (e != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(LBW_ERR_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return hip_fail(e, "hipSetDevice");
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) (void)hipSetDevice(cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return LBW_OK;
}

// The sums of lbw_reduce, over the cells below a horizontal plane of each run
// (plane >= 0) or over all cells (-1), with the partials in `part`
// (nbatch * kReduceBlocks values, then the nbatch sums).
int reduce_on(lbw_handle *h, int32_t what, double *out_host, int plane, int cls, double *part) {
    std::vector<lbw::RunDev> cur(h->nbatch);
    for (int b = 0; b < h->nbatch; ++b) cur[b] = current(h, b);
    hipError_t e = lbw::launch_reduce(h->q, h->precision, cur.data(), h->nbatch, what, h->odd,
                                      part, h->stream, plane, cls);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
    e = hipMemcpyAsync(out_host, part + (size_t)h->nbatch * lbw::kReduceBlocks,
                       sizeof(double) * h->nbatch, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce copy");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce sync");
    for (int b = 0; b < h->nbatch; ++b)
        if (!std::isfinite(out_host[b])) return fail(LBW_ERR_NONFINITE, "run %d: sum is not finite", b);
    return LBW_OK;
}

// The same over the caller's scratch (run 0's buffers).
int reduce_impl(lbw_handle *h, int32_t what, double *out_host, int plane, int cls = -1) {
    size_t need = 0;
    lbw_scratch_bytes(h->cfg.data(), h->nbatch, &need);
    const lbw_buffers &b0 = h->buf[0];
    if (!b0.scratch || b0.scratch_bytes < need)
        return fail(LBW_ERR_INVAL, "scratch of run 0 must hold %zu bytes", need);
    return reduce_on(h, what, out_host, plane, cls, (double *)b0.scratch);
}

int check_reduce(const lbw_handle *h, int32_t what, const double *out_host) {
    if (!h || !out_host) return fail(LBW_ERR_INVAL, "NULL argument");
    if (what < LBW_MASS_C || what > LBW_DEPOSIT) return fail(LBW_ERR_INVAL, "unknown reduction %d", what);
    if (what == LBW_MASS_S && !h->has_s) return fail(LBW_ERR_INVAL, "run has no S");
    if (what == LBW_MASS_FLUID && h->fluid_mode != LBW_FLUID_LBM)
        return fail(LBW_ERR_INVAL, "frozen fluid has no populations");
    return LBW_OK;
}

}  // namespace

int lbw_reduce(lbw_handle *h, int32_t what, double *out_host) {
    const int rc = check_reduce(h, what, out_host);
    return rc ? rc : reduce_impl(h, what, out_host, -1);
}

int lbw_reduce_static(lbw_handle *h, int32_t what, double *out_host) {
    int rc = check_reduce(h, what, out_host);
    if (rc) return rc;
    if (h->nbatch > kStaticRuns)
        return fail(LBW_ERR_INVAL, "lbw_reduce_static handles at most %d runs (got %d)", kStaticRuns,
                    h->nbatch);
    double *p = nullptr;
    if ((rc = static_scratch(h, &p))) return rc;
    // every partial and every sum is written before it is read, so nothing
    // left from an earlier call needs clearing
    return reduce_on(h, what, out_host, -1, -1, p);
}

int lbw_reduce_class(lbw_handle *h, int32_t what, int32_t cls, double *out_host) {
    if (!h || !out_host) return fail(LBW_ERR_INVAL, "NULL argument");
    if (what != LBW_MASS_C && what != LBW_DEPOSIT)
        return fail(LBW_ERR_INVAL, "per-class sums exist for LBW_MASS_C and LBW_DEPOSIT (got %d)", what);
    for (int b = 0; b < h->nbatch; ++b)
        if (cls < 0 || cls >= h->run[b].ncls)
            return fail(LBW_ERR_INVAL, "run %d: class %d outside [0, %d)", b, cls, h->run[b].ncls);
    return reduce_impl(h, what, out_host, -1, cls);
}

int lbw_mass_below(lbw_handle *h, int32_t plane, double *out_host) {
    if (!h || !out_host) return fail(LBW_ERR_INVAL, "NULL argument");
    for (int b = 0; b < h->nbatch; ++b) {
        const lbw::RunDev &r = h->run[b];
        const int nv = h->dim == 2 ? r.ny : r.nz;
        if (plane < 0 || plane > nv)
            return fail(LBW_ERR_INVAL, "run %d: plane %d outside [0, %d]", b, plane, nv);
    }
    return reduce_impl(h, LBW_MASS_C, out_host, plane);
}

int lbw_front_psd(lbw_handle *h, int32_t run, const double *height_dev, int32_t axis,
                  int32_t index, double *out_dev) {
    int rc = check_run(h, run);
    if (rc) return rc;
    if (!height_dev || !out_dev) return fail(LBW_ERR_INVAL, "NULL argument");
    const lbw::RunDev &r = h->run[run];
    if (axis < 0 || axis > h->dim - 2)
        return fail(LBW_ERR_INVAL, "axis %d is not a lateral axis of a %dD run", axis, h->dim);
    const int nslice = axis == 0 ? (h->dim == 3 ? r.ny : 1) : r.nx;
    if (index < -1 || index >= nslice)
        return fail(LBW_ERR_INVAL, "slice index %d outside [-1, %d)", index, nslice);
    hipError_t e = lbw::launch_front_psd(r, h->dim, height_dev, axis, index, out_dev, h->stream);
    return e == hipSuccess ? LBW_OK : hip_fail(e, "front-psd launch");
}

int lbw_front_height(lbw_handle *h, int32_t run, double threshold, double *out_dev) {
    int rc = check_run(h, run);
    if (rc) return rc;
    if (!out_dev) return fail(LBW_ERR_INVAL, "NULL output");
    if (!std::isfinite(threshold)) return fail(LBW_ERR_INVAL, "threshold must be finite");
    hipError_t e = lbw::launch_front_height(h->precision, h->run[run], h->dim, threshold, out_dev, h->stream);
    return e == hipSuccess ? LBW_OK : hip_fail(e, "front-height launch");
}

}  // extern "C"
