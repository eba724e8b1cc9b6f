// Device helpers shared by the HIP sources of libpcg: XCD-aware workgroup
// numbering, deterministic wavefront / grid reductions and the scalar steps
// of the conjugate gradient iteration.
#pragma once

#include "internal.h"

namespace pcg {

// Workgroup b is placed on XCD b % 8 by the dispatcher; renumber so that
// each XCD walks one contiguous range of column tiles and the halo columns
// shared by neighbouring tiles stay in that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    const int64_t q = nb >> 3, r = nb & 7;
    const int64_t x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Block-reduce NV sums, publish them in slot `blk` of `part`, and return
// true in the workgroup that finished last, with the fixed-order totals of
// all `nblk` slots in tot (identical in every thread of that workgroup).
template <int NV>
__device__ __forceinline__ bool reduce_last(double (&v)[NV], double* part, int64_t blk,
                                            int64_t nblk, uint32_t* ticket, double (&tot)[NV])
{
    __shared__ double sm[kBlock / kWave][NV];
    __shared__ int is_last;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sm[wave][i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) s += sm[w][i];
            __hip_atomic_store(&part[blk * kRedSlots + i], s, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        const uint32_t t = atomicAdd(ticket, 1u);
        is_last = (t == (uint32_t)(nblk - 1));
        __threadfence();
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += kBlock) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            acc[i] += __hip_atomic_load(&part[b * kRedSlots + i], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = wave_sum(acc[i]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sm[wave][i] = acc[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) s += sm[w][i];
        tot[i] = s;
    }
    if (threadIdx.x == 0) *ticket = 0u;
    return true;
}

// ----------------------------------------------------------- scalar steps --

// Scalar step after kernel B (Alg. InterleavedPCG): ||r||, exit test, beta.
__device__ inline void finish_prec(SolverState* s, double R, double kappa)
{
    const double rn = sqrt(R);
    if (s->iter == 0) s->r0norm = rn;
    s->rnorm = rn;
    if (!isfinite(rn) || !isfinite(kappa)) { s->flag = kBreakdown; return; }
    if (s->r0norm == 0.0 || rn / s->r0norm < s->rtol || rn < s->atol) { s->flag = kConverged; return; }
    if (s->iter >= s->max_iter) { s->flag = kMaxIter; return; }
    if (!(kappa > 0.0)) { s->flag = kBreakdown; return; }
    s->beta = kappa / s->kappa_old;
    s->kappa_old = kappa;
}

// Scalar step after kernel A: alpha = kappa_old / sigma.
__device__ inline void finish_apply(SolverState* s, double sigma)
{
    if (!(sigma > 0.0) || !isfinite(sigma)) { s->flag = kBreakdown; return; }
    s->sigma = sigma;
    s->alpha = s->kappa_old / sigma;
    s->iter += 1;
}

}  // namespace pcg
