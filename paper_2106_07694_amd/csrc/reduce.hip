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

template <int Q, typename T>
__global__ void __launch_bounds__(256) k_partial(RunDev r, int what, bool odd, bool shifted,
                                                 int plane, double *__restrict__ part) {
    double acc = 0.0;
    int64_t n = (what == LBW_DEPOSIT) ? r.ncol : r.N;
    if (plane >= 0 && (what == LBW_MASS_C || what == LBW_MASS_S) && (int64_t)plane * r.ncol < n)
        n = (int64_t)plane * r.ncol;   // planes are the slowest axis
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        if (what == LBW_MASS_C) {
            acc += (double)((const T *)r.c)[k];
        } else if (what == LBW_MASS_S) {
            acc += (double)((const T *)r.s)[k];
        } else if (what == LBW_MASS_FLUID) {
            using L = Lattice<Q>;
            int x, y, z;
            coords<L::D>(r, k, x, y, z);
            double s = shifted ? 1.0 : 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) s += (double)load_canonical<Q, T>(r, (const T *)r.f, i, k, x, y, z, odd);
            acc += s;
        } else {
            acc += r.dep[k];
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
                    double *scratch, hipStream_t st, int plane) {
    for (int b = 0; b < nbatch; ++b)
        k_partial<Q, T><<<kReduceBlocks, 256, 0, st>>>(runs[b], what, odd, shifted, plane,
                                                        scratch + (int64_t)b * kReduceBlocks);
    k_final<<<nbatch, 256, 0, st>>>(scratch, kReduceBlocks, scratch + (int64_t)nbatch * kReduceBlocks);
    return hipGetLastError();
}

// One thread per bottom column scans upward for the first cell with
// C >= thr (consecutive threads read consecutive cells of a plane) and
// interpolates linearly between the centres of that cell and the one below,
// in double: height (v - 1) + 1/2 + (thr - C_{v-1}) / (C_v - C_{v-1}) from the
// bottom wall; 0 if the bottom cell already holds C >= thr, the domain height
// if no cell does.
template <typename T>
__global__ void __launch_bounds__(256) k_front_height(const T *__restrict__ c, int64_t ncol, int nv,
                                                      double thr, double *__restrict__ out) {
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncol) return;
    double h = (double)nv;
    double below = 0.0;
    for (int v = 0; v < nv; ++v) {
        const double cv = (double)c[col + (int64_t)v * ncol];
        if (cv >= thr) {
            h = v == 0 ? 0.0 : (double)(v - 1) + 0.5 + (thr - below) / (cv - below);
            break;
        }
        below = cv;
    }
    out[col] = h;
}

}  // namespace

hipError_t launch_reduce(int q, int precision, const RunDev *runs, int nbatch, int what, bool odd,
                         double *scratch, hipStream_t st, int plane) {
    const bool sh = precision != LBW_FP64;
    if (precision == LBW_FP32_SHIFTED)
        return q == 9 ? reduce_t<9, float>(runs, nbatch, what, odd, sh, scratch, st, plane)
                      : reduce_t<19, float>(runs, nbatch, what, odd, sh, scratch, st, plane);
    return q == 9 ? reduce_t<9, double>(runs, nbatch, what, odd, sh, scratch, st, plane)
                  : reduce_t<19, double>(runs, nbatch, what, odd, sh, scratch, st, plane);
}

hipError_t launch_front_height(int precision, const RunDev &r, int dim, double thr, double *out,
                               hipStream_t st) {
    const int nv = dim == 2 ? r.ny : r.nz;
    const unsigned grid = (unsigned)((r.ncol + 255) / 256);
    if (precision == LBW_FP32_SHIFTED)
        k_front_height<float><<<grid, 256, 0, st>>>((const float *)r.c, r.ncol, nv, thr, out);
    else
        k_front_height<double><<<grid, 256, 0, st>>>((const double *)r.c, r.ncol, nv, thr, out);
    return hipGetLastError();
}

namespace {

// Power spectral density of a front height along one lateral axis (the
// spectrum whose growth the paper fits against linear stability, eq. 45-46):
// Gamma(k) = |sum_j H_j exp(-2 pi i k j / L)|^2 / (kS L), kS = 1, averaged
// over slices s0 .. s1-1.  One block per wavenumber; each slice's transform
// is a block-wide sum in a fixed order (the same bits on every call), with
// the phase k j reduced modulo L exactly before the sine and cosine.
__global__ void __launch_bounds__(256) k_front_psd(const double *__restrict__ h, int len,
                                                   int64_t step, int64_t stride, int s0, int s1,
                                                   double *__restrict__ out) {
    __shared__ double wre[4], wim[4];
    const int64_t k = blockIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const double two_over_len = 2.0 / (double)len;
    double acc = 0.0;
    for (int s = s0; s < s1; ++s) {
        const double *row = h + (int64_t)s * stride;
        double re = 0.0, im = 0.0;
        for (int j = threadIdx.x; j < len; j += blockDim.x) {
            const int64_t m = (k * j) % len;
            double sn, cs;
            sincospi((double)m * two_over_len, &sn, &cs);   // angle 2 pi m / L
            const double hj = row[(int64_t)j * step];
            re += hj * cs;
            im -= hj * sn;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            re += __shfl_down(re, off, 64);
            im += __shfl_down(im, off, 64);
        }
        if (lane == 0) {
            wre[wid] = re;
            wim[wid] = im;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double tr = 0.0, ti = 0.0;
            for (int i = 0; i < 4; ++i) {
                tr += wre[i];
                ti += wim[i];
            }
            acc += (tr * tr + ti * ti) / (double)len;
        }
        __syncthreads();   // the next slice overwrites wre / wim
    }
    if (threadIdx.x == 0) out[k] = acc / (double)(s1 - s0);
}

}  // namespace

hipError_t launch_front_psd(const RunDev &r, int dim, const double *h, int axis, int index,
                            double *out, hipStream_t st) {
    int len, nslice;
    int64_t step, stride;
    if (axis == 0) {            // rows along x, one per y
        len = r.nx;
        nslice = dim == 3 ? r.ny : 1;
        step = 1;
        stride = r.nx;
    } else {                    // rows along y, one per x
        len = r.ny;
        nslice = r.nx;
        step = r.nx;
        stride = 1;
    }
    const int s0 = index < 0 ? 0 : index, s1 = index < 0 ? nslice : index + 1;
    k_front_psd<<<(unsigned)(len / 2 + 1), 256, 0, st>>>(h, len, step, stride, s0, s1, out);
    return hipGetLastError();
}

}  // namespace lbw
