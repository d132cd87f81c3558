// reduce.hip -- FP64 global sums of a run: particle mass sum C, sugar sum S,
// fluid mass sum rho and the deposited mass m_b (section 4.2.3: mass of
// particles per cell and mass accumulated at the bottom).  Each block
// accumulates a grid-stride slice in double, reduces it across the wavefront
// with shuffles and across waves through LDS, and writes one partial; a
// single block per run then adds the partials in a fixed order.  The result
// does not depend on timing: the same inputs give the same bits.
//
// Also the in-situ diagnostics of the paper's analysis: the mass below a
// horizontal plane (a prefix of the node order, whose change over time is the
// particle mass flux through the plane) and the front of the particle field
// per column (lowest height where C reaches a threshold).
#include "lbm_device.h"

#include <climits>

namespace lbw {
namespace {

__device__ __forceinline__ double block_sum(double acc) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    __shared__ double waves[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) waves[wid] = acc;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) t += waves[i];
    }
    return t;
}

// Sum of x[0 .. n-1] over a grid-stride slice with four independent
// accumulators (four loads in flight per thread), combined in a fixed order.
template <typename V>
__device__ __forceinline__ double strided_sum(const V *__restrict__ x, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (; k + 3 * stride < n; k += 4 * stride) {
        a0 += (double)x[k];
        a1 += (double)x[k + stride];
        a2 += (double)x[k + 2 * stride];
        a3 += (double)x[k + 3 * stride];
    }
    for (; k < n; k += stride) a0 += (double)x[k];
    return (a0 + a1) + (a2 + a3);
}

// cls >= 0: MASS_C and DEPOSIT of that size class only; -1: every class.
template <int Q, typename T>
__global__ void __launch_bounds__(1024) k_partial(RunDev r, int what, bool odd, bool shifted,
                                                  int plane, int cls, double *__restrict__ part) {
    double acc = 0.0;
    const int c0 = cls < 0 ? 0 : cls, c1 = cls < 0 ? r.ncls : cls + 1;
    // the deposit counters of the size classes are contiguous
    int64_t n = (what == LBW_DEPOSIT) ? r.ncol * (c1 - c0) : r.N;
    if (plane >= 0 && (what == LBW_MASS_C || what == LBW_MASS_S) && (int64_t)plane * r.ncol < n)
        n = (int64_t)plane * r.ncol;   // planes are the slowest axis
    if (what == LBW_MASS_C) {
        for (int i = c0; i < c1; ++i) acc += strided_sum((const T *)r.c + (int64_t)i * r.N, n);
    } else if (what == LBW_MASS_S) {
        acc = strided_sum((const T *)r.s, n);
    } else if (what == LBW_DEPOSIT) {
        acc = strided_sum(r.dep + (int64_t)c0 * r.ncol, n);
    } else {
        using L = Lattice<Q>;
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
            int x, y, z;
            coords<L::D>(r, k, x, y, z);
            double s = shifted ? 1.0 : 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) s += (double)load_canonical<Q, T>(r, (const T *)r.f, i, k, x, y, z, odd);
            acc += s;
        }
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_final(const double *__restrict__ part, int nblocks,
                                               double *__restrict__ out) {
    const double *p = part + (int64_t)blockIdx.x * nblocks;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) acc += p[i];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

template <int Q, typename T>
hipError_t reduce_t(const RunDev *runs, int nbatch, int what, bool odd, bool shifted,
                    double *scratch, hipStream_t st, int plane, int cls) {
    for (int b = 0; b < nbatch; ++b)
        k_partial<Q, T><<<kReduceBlocks, 1024, 0, st>>>(runs[b], what, odd, shifted, plane, cls,
                                                        scratch + (int64_t)b * kReduceBlocks);
    k_final<<<nbatch, 256, 0, st>>>(scratch, kReduceBlocks, scratch + (int64_t)nbatch * kReduceBlocks);
    return hipGetLastError();
}

// Front of the particle field: for each bottom column, the first cell v
// (from the bottom wall) with C >= thr, and linear interpolation between the
// centres of that cell and the one below, in double: height (v - 1) + 1/2 +
// (thr - C_{v-1}) / (C_v - C_{v-1}); 0 if the bottom cell already holds
// C >= thr, the domain height if no cell does.
//
// A block owns 64 consecutive columns (a wave reads 64 consecutive cells of
// a plane) and climbs them in rounds of W * U cells: wave w loads cells
// [base + w U, base + (w + 1) U) of its lane's column, U independent loads in
// flight, and the lowest hit of the round over the W waves ends the column.
// The scan thus stops within one round of the front, with W * U loads per
// column in flight instead of one dependent load at a time.
//
// With several particle size classes (MULTI) C is their total, summed in
// FP64 in class order; c then holds ncls fields of N values.
template <typename T, int W, int U, bool MULTI>
__global__ void __launch_bounds__(64 * W) k_front_height(const T *__restrict__ c, int64_t ncol,
                                                         int nv, int ncls, int64_t N, double thr,
                                                         double *__restrict__ out) {
    __shared__ int hit[W][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.x * 64 + lane;
    bool done = col >= ncol;                 // the same in every wave of the block
    for (int base = 0; base < nv; base += W * U) {
        int first = INT_MAX;
        if (!done) {
            const int v0 = base + w * U;
            double cv[U];
            // unconditional loads (the index clamped into the column): a
            // guarded load would make the compiler wait for each one in turn
#pragma unroll
            for (int u = 0; u < U; ++u) cv[u] = (double)c[col + (int64_t)min(v0 + u, nv - 1) * ncol];
            if constexpr (MULTI) {
                for (int i = 1; i < ncls; ++i) {
                    const T *ci = c + (int64_t)i * N;
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        cv[u] += (double)ci[col + (int64_t)min(v0 + u, nv - 1) * ncol];
                }
            }
#pragma unroll
            for (int u = U - 1; u >= 0; --u)
                if (v0 + u < nv && cv[u] >= thr) first = v0 + u;
        }
        hit[w][lane] = first;
        __syncthreads();
        int v = INT_MAX;
#pragma unroll
        for (int i = 0; i < W; ++i) v = min(v, hit[i][lane]);
        if (!done && v != INT_MAX) {
            if (w == 0) {
                double h = 0.0;
                if (v > 0) {
                    double cv = (double)c[col + (int64_t)v * ncol];
                    double cb = (double)c[col + (int64_t)(v - 1) * ncol];
                    if constexpr (MULTI) {
                        for (int i = 1; i < ncls; ++i) {
                            cv += (double)c[(int64_t)i * N + col + (int64_t)v * ncol];
                            cb += (double)c[(int64_t)i * N + col + (int64_t)(v - 1) * ncol];
                        }
                    }
                    h = (double)(v - 1) + 0.5 + (thr - cb) / (cv - cb);
                }
                out[col] = h;
            }
            done = true;
        }
        // also orders this round's reads of hit[] before the next round's writes
        if (__syncthreads_and(done)) return;
    }
    if (!done && w == 0) out[col] = (double)nv;
}

}  // namespace

hipError_t launch_reduce(int q, int precision, const RunDev *runs, int nbatch, int what, bool odd,
                         double *scratch, hipStream_t st, int plane, int cls) {
    const bool sh = precision != LBW_FP64;
    if (precision == LBW_FP32_SHIFTED)
        return q == 9 ? reduce_t<9, float>(runs, nbatch, what, odd, sh, scratch, st, plane, cls)
                      : reduce_t<19, float>(runs, nbatch, what, odd, sh, scratch, st, plane, cls);
    return q == 9 ? reduce_t<9, double>(runs, nbatch, what, odd, sh, scratch, st, plane, cls)
                  : reduce_t<19, double>(runs, nbatch, what, odd, sh, scratch, st, plane, cls);
}

template <typename T, bool MULTI>
static void front_height_t(const T *c, int64_t ncol, int nv, int ncls, int64_t N, double thr,
                           double *out, hipStream_t st) {
    const unsigned grid = (unsigned)((ncol + 63) / 64);
    // few columns (2D grids): more waves per column keep enough loads in flight
    if (ncol >= 16384)
        k_front_height<T, 4, 16, MULTI><<<grid, 256, 0, st>>>(c, ncol, nv, ncls, N, thr, out);
    else
        k_front_height<T, 16, 8, MULTI><<<grid, 1024, 0, st>>>(c, ncol, nv, ncls, N, thr, out);
}

template <typename T>
static void front_height_c(const RunDev &r, int nv, double thr, double *out, hipStream_t st) {
    if (r.ncls > 1)
        front_height_t<T, true>((const T *)r.c, r.ncol, nv, r.ncls, r.N, thr, out, st);
    else
        front_height_t<T, false>((const T *)r.c, r.ncol, nv, 1, r.N, thr, out, st);
}

hipError_t launch_front_height(int precision, const RunDev &r, int dim, double thr, double *out,
                               hipStream_t st) {
    const int nv = dim == 2 ? r.ny : r.nz;
    if (precision == LBW_FP32_SHIFTED)
        front_height_c<float>(r, nv, thr, out, st);
    else
        front_height_c<double>(r, nv, thr, out, st);
    return hipGetLastError();
}

namespace {

// Power spectral density of a front height along one lateral axis (the
// spectrum whose growth the paper fits against linear stability, eq. 45-46):
// Gamma(k) = |sum_j H_j exp(-2 pi i k j / L)|^2 / (kS L), kS = 1, averaged
// over rows s0 .. s1-1.  One block of four waves per wavenumber k.  The
// twiddles exp(-2 pi i k j / L), with the phase k j reduced modulo L exactly,
// are tabulated once per block in LDS when the row fits (L <= kPsdTable).
// Every sum runs in a fixed order, so the same input gives the same bits.
constexpr int kPsdTable = 2048;   // 32 KiB of LDS

template <bool TABLE>
__device__ __forceinline__ void twiddle(const double *tw, int64_t k, int j, int len, double &cs,
                                        double &sn) {
    if constexpr (TABLE) {
        cs = tw[2 * j];
        sn = tw[2 * j + 1];
    } else {
        sincospi((double)((k * j) % len) * (2.0 / (double)len), &sn, &cs);
    }
}

template <bool TABLE>
__device__ __forceinline__ void fill_twiddles(double *tw, int64_t k, int len) {
    if constexpr (TABLE) {
        for (int j = threadIdx.x; j < len; j += blockDim.x)
            sincospi((double)((k * j) % len) * (2.0 / (double)len), &tw[2 * j + 1], &tw[2 * j]);
        __syncthreads();
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Few rows: one wave per row, lanes over its samples (element j of row s at
// h[s * row_stride + j * step]).
template <bool TABLE>
__global__ void __launch_bounds__(256) k_front_psd_waves(const double *__restrict__ h, int len,
                                                         int64_t row_stride, int64_t step, int s0,
                                                         int s1, double *__restrict__ out) {
    extern __shared__ double tw[];
    __shared__ double wsum[4];
    const int64_t k = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    fill_twiddles<TABLE>(tw, k, len);
    double acc = 0.0;
    for (int s = s0 + w; s < s1; s += 4) {
        const double *row = h + (int64_t)s * row_stride;
        double re = 0.0, im = 0.0;
        for (int j = lane; j < len; j += 64) {
            double cs, sn;
            twiddle<TABLE>(tw, k, j, len, cs, sn);
            const double hj = row[(int64_t)j * step];
            re += hj * cs;
            im -= hj * sn;
        }
        re = wave_sum(re);
        im = wave_sum(im);
        acc += (re * re + im * im) / (double)len;    // meaningful in lane 0
    }
    if (lane == 0) wsum[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[k] = (wsum[0] + wsum[1] + wsum[2] + wsum[3]) / (double)(s1 - s0);
}

// Many rows: one lane per row, each lane walking its own row with the
// twiddle of sample j broadcast from LDS; no cross-lane sum per row.  Along
// y (rows one per x) a wave reads 64 consecutive values per sample.
template <bool TABLE>
__global__ void __launch_bounds__(256) k_front_psd_lanes(const double *__restrict__ h, int len,
                                                         int64_t row_stride, int64_t step, int s0,
                                                         int s1, double *__restrict__ out) {
    extern __shared__ double tw[];
    __shared__ double wsum[4];
    const int64_t k = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    fill_twiddles<TABLE>(tw, k, len);
    double acc = 0.0;
    for (int sb = s0 + 64 * w; sb < s1; sb += 256) {
        const int s = sb + lane;
        if (s < s1) {
            const double *row = h + (int64_t)s * row_stride;
            double re = 0.0, im = 0.0;
            for (int j = 0; j < len; ++j) {
                double cs, sn;
                twiddle<TABLE>(tw, k, j, len, cs, sn);
                const double hj = row[(int64_t)j * step];
                re += hj * cs;
                im -= hj * sn;
            }
            acc += (re * re + im * im) / (double)len;
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) wsum[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[k] = (wsum[0] + wsum[1] + wsum[2] + wsum[3]) / (double)(s1 - s0);
}

}  // namespace

hipError_t launch_front_psd(const RunDev &r, int dim, const double *h, int axis, int index,
                            double *out, hipStream_t st) {
    // along x: rows one per y, samples contiguous; along y: rows one per x,
    // samples nx apart
    const int len = axis == 0 ? r.nx : r.ny;
    const int nslice = axis == 0 ? (dim == 3 ? r.ny : 1) : r.nx;
    const int64_t row_stride = axis == 0 ? r.nx : 1, step = axis == 0 ? 1 : r.nx;
    const int s0 = index < 0 ? 0 : index, s1 = index < 0 ? nslice : index + 1;
    const unsigned grid = (unsigned)(len / 2 + 1);
    const bool table = len <= kPsdTable;
    const size_t lds = table ? (size_t)len * 2 * sizeof(double) : 0;
    const bool lanes = s1 - s0 >= 64;
    if (lanes && table)
        k_front_psd_lanes<true><<<grid, 256, lds, st>>>(h, len, row_stride, step, s0, s1, out);
    else if (lanes)
        k_front_psd_lanes<false><<<grid, 256, 0, st>>>(h, len, row_stride, step, s0, s1, out);
    else if (table)
        k_front_psd_waves<true><<<grid, 256, lds, st>>>(h, len, row_stride, step, s0, s1, out);
    else
        k_front_psd_waves<false><<<grid, 256, 0, st>>>(h, len, row_stride, step, s0, s1, out);
    return hipGetLastError();
}

}  // namespace lbw
