// lbm.hip -- lattice-Boltzmann part of the coupled step: moments with the
// Guo half-force shift (eq. 19-20, 22), BGK collision with Guo forcing
// (eq. 18, 22) and streaming with half-way bounce-back (section 2.3.1),
// done in place with the two-kernel "AA" access pattern:
//
//  even step: node k reads its own populations from slot i and writes the
//             post-collision value f*_i into slot opp(i) of the same node;
//  odd step:  node k gathers f_i from slot opp(i) of node k - c_i (the value
//             the even step left there), or, when k - c_i lies beyond a wall,
//             its own slot i (bounce-back, plus the moving-wall term), then
//             scatters f*_i into slot i of node k + c_i, or into its own slot
//             opp(i) when k + c_i lies beyond a wall.
//
// Every memory location is read and written by the same thread within a
// step, so one buffer suffices and no synchronisation is needed.  Both kernels
// move exactly 2Q values per node: the traffic of a two-lattice scheme at
// half the footprint.  The node velocity u^n is written for the transport
// kernels, which use it frozen over the three RK stages.
#include "lbm_device.h"

namespace lbw {
namespace {

template <int Q, typename T, bool SH, bool ODD, bool NT>
__device__ __forceinline__ void collide_stream_node(const RunDev &r, int64_t k) {
    using L = Lattice<Q>;
    constexpr int D = L::D;
    T *__restrict__ f = (T *)r.f;
    int x, y, z;
    coords<D>(r, k, x, y, z);

    T fi[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) fi[i] = load_canonical<Q, T, NT>(r, f, i, k, x, y, z, ODD);

    // moments (eq. 19-20) with the Guo shift and the buoyancy force (eq. 10),
    // then the BGK + Guo collision (eq. 18, 22)
    T F[3], uu[3], rho;
    lbm_force<D, T>(r, (const T *)r.c, (const T *)r.s, k, F);
    lbm_collide<Q, T, SH>(r, fi, F, rho, uu);
    T *__restrict__ uo = (T *)r.u;
    uo[k] = uu[0];
    uo[r.N + k] = uu[1];
    if (D == 3) uo[2 * r.N + k] = uu[2];
    if (r.rho) ((T *)r.rho)[k] = rho;

    // store (streaming)
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (!ODD) {
            pop_store<T, NT>(&f[(int64_t)L::opp[i] * r.N + k], fi[i]);
        } else {
            const int64_t dst = displaced<D>(r, x, y, z, L::cx[i], L::cy[i], L::cz[i]);
            if (dst >= 0) {
                pop_store<T, NT>(&f[(int64_t)i * r.N + dst], fi[i]);
            } else {
                T v = fi[i];
                if (dst == -2) v -= (T)lid_term<Q>(r, i);
                pop_store<T, NT>(&f[(int64_t)L::opp[i] * r.N + k], v);
            }
        }
    }
}

// Every node of one run, one per thread.
template <int Q, typename T, bool SH, bool ODD, bool NT>
__global__ void __launch_bounds__(1024) k_collide_stream(RunDev r) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r.N) return;
    collide_stream_node<Q, T, SH, ODD, NT>(r, k);
}

// Batched form: a persistent grid walks the thread blocks of every run;
// blk_start[b] is the first block of run b (prefix sum, nbatch + 1 entries).
template <int Q, typename T, bool SH, bool ODD, bool NT>
__global__ void __launch_bounds__(1024) k_collide_stream_batched(const RunDev *__restrict__ runs,
                                                                 const int *__restrict__ blk_start,
                                                                 int nbatch, int sflip) {
    const int total = blk_start[nbatch];
    int b = 0;
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        while (blk_start[b + 1] <= w) ++b;   // w only grows, so b only grows
        RunDev r = runs[b];
        if (sflip) { void *t = r.s; r.s = r.s2; r.s2 = t; }
        const int64_t k = (int64_t)(w - blk_start[b]) * blockDim.x + threadIdx.x;
        if (k < r.N) collide_stream_node<Q, T, SH, ODD, NT>(r, k);
    }
}

template <int Q, typename T, bool SH>
__global__ void k_equilibrium(RunDev r, bool odd, const T *__restrict__ rho_in,
                              const T *__restrict__ u_in) {
    using L = Lattice<Q>;
    constexpr int D = L::D;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r.N) return;
    int x, y, z;
    coords<D>(r, k, x, y, z);
    const T rho = rho_in ? rho_in[k] : (T)1;
    T ux = 0, uy = 0, uz = 0;
    if (u_in) {
        ux = u_in[k];
        uy = u_in[r.N + k];
        if (D == 3) uz = u_in[2 * r.N + k];
    }
    const T usq = ux * ux + uy * uy + uz * uz;
    T *__restrict__ f = (T *)r.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T w = (T)L::w[i];
        const T cu = (T)L::cx[i] * ux + (T)L::cy[i] * uy + (T)L::cz[i] * uz;
        const T poly = (T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * usq;
        const T v = SH ? w * ((rho - (T)1) + rho * poly) : w * rho * ((T)1 + poly);
        store_canonical<Q, T>(r, f, i, k, x, y, z, odd, v);
    }
}

template <int Q, typename T>
__global__ void k_import_f(RunDev r, const T *__restrict__ src) {
    using L = Lattice<Q>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r.N) return;
    int x, y, z;
    coords<L::D>(r, k, x, y, z);
    T *__restrict__ f = (T *)r.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) store_canonical<Q, T>(r, f, i, k, x, y, z, true, src[(int64_t)i * r.N + k]);
}

template <int Q, typename T>
__global__ void k_export_f(RunDev r, T *__restrict__ dst) {
    using L = Lattice<Q>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r.N) return;
    int x, y, z;
    coords<L::D>(r, k, x, y, z);
    const T *__restrict__ f = (const T *)r.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) dst[(int64_t)i * r.N + k] = load_canonical<Q, T>(r, f, i, k, x, y, z, true);
}

inline unsigned blocks_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Populations beyond this size are streamed with non-temporal accesses: they
// cannot stay in the 256 MB last-level (Infinity) cache between steps, and
// bypassing it measured 6% faster for 2.5 GB; smaller sets (which do stay
// there) measured 15% slower that way.
constexpr size_t kStreamingBytes = (size_t)192 << 20;
inline bool streaming_populations(size_t bytes) { return bytes > kStreamingBytes; }

template <int Q, typename T, bool SH>
hipError_t collide_stream_t(const RunDev &r, bool odd, int block, hipStream_t st) {
    const bool nt = streaming_populations((size_t)Q * sizeof(T) * (size_t)r.N);
    const dim3 grid(blocks_for(r.N, block));
    if (odd) {
        if (nt) k_collide_stream<Q, T, SH, true, true><<<grid, block, 0, st>>>(r);
        else k_collide_stream<Q, T, SH, true, false><<<grid, block, 0, st>>>(r);
    } else {
        if (nt) k_collide_stream<Q, T, SH, false, true><<<grid, block, 0, st>>>(r);
        else k_collide_stream<Q, T, SH, false, false><<<grid, block, 0, st>>>(r);
    }
    return hipGetLastError();
}

template <int Q, typename T, bool SH>
hipError_t collide_stream_batched_t(const RunDev *runs, const int *blk_start, int nbatch, int sflip,
                                    bool odd, int block, int grid, int64_t nodes, hipStream_t st) {
    const bool nt = streaming_populations((size_t)Q * sizeof(T) * (size_t)nodes);
    if (odd) {
        if (nt) k_collide_stream_batched<Q, T, SH, true, true><<<grid, block, 0, st>>>(runs, blk_start, nbatch, sflip);
        else k_collide_stream_batched<Q, T, SH, true, false><<<grid, block, 0, st>>>(runs, blk_start, nbatch, sflip);
    } else {
        if (nt) k_collide_stream_batched<Q, T, SH, false, true><<<grid, block, 0, st>>>(runs, blk_start, nbatch, sflip);
        else k_collide_stream_batched<Q, T, SH, false, false><<<grid, block, 0, st>>>(runs, blk_start, nbatch, sflip);
    }
    return hipGetLastError();
}

template <int Q>
hipError_t collide_stream_q(int precision, const RunDev &r, bool odd, int block, hipStream_t st) {
    switch (precision) {
        case LBW_FP64: return collide_stream_t<Q, double, false>(r, odd, block, st);
        case LBW_FP64_SHIFTED: return collide_stream_t<Q, double, true>(r, odd, block, st);
        case LBW_FP32_SHIFTED: return collide_stream_t<Q, float, true>(r, odd, block, st);
    }
    return hipErrorInvalidValue;
}

template <int Q>
hipError_t equilibrium_q(int precision, const RunDev &r, bool odd, const void *rho, const void *u,
                         hipStream_t st) {
    const int block = 256;
    const dim3 grid(blocks_for(r.N, block));
    switch (precision) {
        case LBW_FP64:
            k_equilibrium<Q, double, false><<<grid, block, 0, st>>>(r, odd, (const double *)rho, (const double *)u);
            break;
        case LBW_FP64_SHIFTED:
            k_equilibrium<Q, double, true><<<grid, block, 0, st>>>(r, odd, (const double *)rho, (const double *)u);
            break;
        case LBW_FP32_SHIFTED:
            k_equilibrium<Q, float, true><<<grid, block, 0, st>>>(r, odd, (const float *)rho, (const float *)u);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int Q>
hipError_t import_q(int precision, const RunDev &r, const void *src, hipStream_t st) {
    const int block = 256;
    const dim3 grid(blocks_for(r.N, block));
    if (precision == LBW_FP32_SHIFTED)
        k_import_f<Q, float><<<grid, block, 0, st>>>(r, (const float *)src);
    else
        k_import_f<Q, double><<<grid, block, 0, st>>>(r, (const double *)src);
    return hipGetLastError();
}

template <int Q>
hipError_t export_q(int precision, const RunDev &r, void *dst, hipStream_t st) {
    const int block = 256;
    const dim3 grid(blocks_for(r.N, block));
    if (precision == LBW_FP32_SHIFTED)
        k_export_f<Q, float><<<grid, block, 0, st>>>(r, (float *)dst);
    else
        k_export_f<Q, double><<<grid, block, 0, st>>>(r, (double *)dst);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_collide_stream(int q, int precision, const RunDev &r, bool odd, int block,
                                 hipStream_t st) {
    if (block <= 0 || block > 1024 || block % 64) return hipErrorInvalidValue;
    if (r.N <= 0) return hipSuccess;
    return q == 9 ? collide_stream_q<9>(precision, r, odd, block, st)
                  : collide_stream_q<19>(precision, r, odd, block, st);
}

hipError_t launch_collide_stream_batched(int q, int precision, const RunDev *runs, const int *blk_start,
                                         int nbatch, int sflip, bool odd, int block, int grid,
                                         int64_t nodes, hipStream_t st) {
    if (block <= 0 || block > 1024 || block % 64 || grid <= 0) return hipErrorInvalidValue;
    switch (precision) {
        case LBW_FP64:
            return q == 9 ? collide_stream_batched_t<9, double, false>(runs, blk_start, nbatch, sflip, odd, block, grid, nodes, st)
                          : collide_stream_batched_t<19, double, false>(runs, blk_start, nbatch, sflip, odd, block, grid, nodes, st);
        case LBW_FP64_SHIFTED:
            return q == 9 ? collide_stream_batched_t<9, double, true>(runs, blk_start, nbatch, sflip, odd, block, grid, nodes, st)
                          : collide_stream_batched_t<19, double, true>(runs, blk_start, nbatch, sflip, odd, block, grid, nodes, st);
        case LBW_FP32_SHIFTED:
            return q == 9 ? collide_stream_batched_t<9, float, true>(runs, blk_start, nbatch, sflip, odd, block, grid, nodes, st)
                          : collide_stream_batched_t<19, float, true>(runs, blk_start, nbatch, sflip, odd, block, grid, nodes, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_equilibrium(int q, int precision, const RunDev &r, bool odd, const void *rho,
                              const void *u, hipStream_t st) {
    return q == 9 ? equilibrium_q<9>(precision, r, odd, rho, u, st)
                  : equilibrium_q<19>(precision, r, odd, rho, u, st);
}

hipError_t launch_import_f(int q, int precision, const RunDev &r, bool odd, const void *src,
                           hipStream_t st) {
    if (!odd) {
        const size_t es = precision == LBW_FP32_SHIFTED ? 4 : 8;
        return hipMemcpyAsync(r.f, src, (size_t)q * r.N * es, hipMemcpyDeviceToDevice, st);
    }
    return q == 9 ? import_q<9>(precision, r, src, st) : import_q<19>(precision, r, src, st);
}

hipError_t launch_export_f(int q, int precision, const RunDev &r, bool odd, void *dst,
                           hipStream_t st) {
    if (!odd) {
        const size_t es = precision == LBW_FP32_SHIFTED ? 4 : 8;
        return hipMemcpyAsync(dst, r.f, (size_t)q * r.N * es, hipMemcpyDeviceToDevice, st);
    }
    return q == 9 ? export_q<9>(precision, r, dst, st) : export_q<19>(precision, r, dst, st);
}

}  // namespace lbw
