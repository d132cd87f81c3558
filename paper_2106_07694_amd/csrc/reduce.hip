// reduce.hip -- FP64 global sums of a run: particle mass sum C, sugar sum S,
// fluid mass sum rho and the deposited mass m_b (section 4.2.3: mass of
// particles per cell and mass accumulated at the bottom).  Each block
// accumulates a grid-stride slice in double, reduces it across the wavefront
// with shuffles and across waves through LDS, and writes one partial; a
// single block per run then adds the partials in a fixed order.  The result
// does not depend on timing: the same inputs give the same bits.
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
                                                 double *__restrict__ part) {
    double acc = 0.0;
    const int64_t n = (what == LBW_DEPOSIT) ? r.ncol : r.N;
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
                    double *scratch, hipStream_t st) {
    for (int b = 0; b < nbatch; ++b)
        k_partial<Q, T><<<kReduceBlocks, 256, 0, st>>>(runs[b], what, odd, shifted,
                                                        scratch + (int64_t)b * kReduceBlocks);
    k_final<<<nbatch, 256, 0, st>>>(scratch, kReduceBlocks, scratch + (int64_t)nbatch * kReduceBlocks);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_reduce(int q, int precision, const RunDev *runs, int nbatch, int what, bool odd,
                         double *scratch, hipStream_t st) {
    const bool sh = precision != LBW_FP64;
    if (precision == LBW_FP32_SHIFTED)
        return q == 9 ? reduce_t<9, float>(runs, nbatch, what, odd, sh, scratch, st)
                      : reduce_t<19, float>(runs, nbatch, what, odd, sh, scratch, st);
    return q == 9 ? reduce_t<9, double>(runs, nbatch, what, odd, sh, scratch, st)
                  : reduce_t<19, double>(runs, nbatch, what, odd, sh, scratch, st);
}

}  // namespace lbw
