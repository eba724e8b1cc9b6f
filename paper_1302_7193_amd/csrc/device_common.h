// Device helpers shared by the HIP sources of libpcg: XCD-aware workgroup
// numbering, deterministic wavefront / grid reductions and the scalar steps
// of the conjugate gradient iteration.
#pragma once

#include <type_traits>

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

// ------------------------------------------------------ cross-lane moves --
// DPP controls (GFX9): row_shr:d / row_shl:d move within rows of 16 lanes,
// wave_shr:1 / wave_shl:1 across the whole wavefront by one lane.  A lane
// reads another lane's register directly, without the LDS round trip of a
// permute.
constexpr int kRowShr = 0x110, kRowShl = 0x100, kWaveShr1 = 0x138, kWaveShl1 = 0x130;
// quad_perm [1,0,3,2] and [2,3,0,1]; row_ror:n rotates within a row by n.
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kRowRor = 0x120;

// Lane i receives x from the lane CTRL names; lanes without a source lane
// (past the row or wavefront edge) receive the identity ONE ? 1 : 0.  A
// 32-bit half whose identity bits are zero is moved with the zero fill for
// missing source lanes (bound_ctrl), so its destination needs no
// initialisation; only the high half of a floating-point 1 keeps an old
// value.
template <int CTRL>
__device__ __forceinline__ int dpp_half(int x, int id_bits)
{
    if (id_bits == 0) return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true);
    return __builtin_amdgcn_update_dpp(id_bits, x, CTRL, 0xF, 0xF, false);
}

template <int CTRL, int ONE = 0, typename T>
__device__ __forceinline__ T dpp_move(T x)
{
    static_assert(ONE == 0 || ONE == 1, "identity 0 or 1");
    if constexpr (sizeof(T) == 8) {
        const int64_t xb = __builtin_bit_cast(int64_t, x);
        const int64_t ib = ONE ? __builtin_bit_cast(int64_t, T(1)) : 0;
        const int lo = dpp_half<CTRL>((int)xb, (int)ib);
        const int hi = dpp_half<CTRL>((int)(xb >> 32), (int)(ib >> 32));
        return __builtin_bit_cast(T, ((int64_t)hi << 32) | (int64_t)(uint32_t)lo);
    } else {
        const int ib = ONE ? __builtin_bit_cast(int, T(1)) : 0;
        return __builtin_bit_cast(T, dpp_half<CTRL>(__builtin_bit_cast(int, x), ib));
    }
}

// The value of x in lane `lane` (a constant), as a wavefront-uniform value.
template <typename T>
__device__ __forceinline__ T read_lane(T x, int lane)
{
    if constexpr (sizeof(T) == 8) {
        const int64_t xb = __builtin_bit_cast(int64_t, x);
        const int lo = __builtin_amdgcn_readlane((int)xb, lane);
        const int hi = __builtin_amdgcn_readlane((int)(xb >> 32), lane);
        return __builtin_bit_cast(T, ((int64_t)hi << 32) | (int64_t)(uint32_t)lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
    }
}

// Sum over the wavefront in a fixed order, the same bits in every lane:
// within each row of 16 lanes a quad butterfly and rotations by 4 and 8
// lanes (lane 0 of a row ends with ((q0 + q1) + (q2 + q3)) of its quads'
// sums), then the four rows' sums from lanes 0, 16, 32, 48.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_move<kQuadXor1>(v);
    v += dpp_move<kQuadXor2>(v);
    v += dpp_move<kRowRor + 4>(v);
    v += dpp_move<kRowRor + 8>(v);
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum NV per-thread values over the workgroup in a fixed order; the totals
// are returned in every thread.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (&out)[NV])
{
    __shared__ double sm[kBlock / kWave][NV];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sm[wave][i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) s += sm[w][i];
        out[i] = s;
    }
    __syncthreads();
}

// Fixed-order total of the nblk published partial sums, computed as if by
// kFinalThreads virtual threads.  The slots are read in 16-byte steps (two
// slots of a one-value reduction, one slot of a two-value one): virtual
// thread v adds steps v, v + 1024, ... in order (a step's slots in order),
// virtual wavefronts add their 64 lanes by shuffles, and the 16 wavefront
// sums are added in order.  A workgroup of BS threads plays 1024 / BS
// virtual threads per thread, so the finalize launch (1024 threads) and the
// in-kernel mode (256 threads) produce identical bits.  Every thread gets
// the totals.  COHERENT: device-scope atomic loads (partials written by
// other workgroups of the running kernel).
constexpr int kFinalThreads = 1024;

template <int NV, bool COHERENT, int BS>
__device__ __forceinline__ void sum_partials(const double* part, int64_t nblk, double (&tot)[NV])
{
    constexpr int R = kFinalThreads / BS;
    constexpr int kWavesV = kFinalThreads / kWave;
    constexpr int S = 2 / NV;          // slots per 16-byte step
    __shared__ double sm[kWavesV][NV];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t full = nblk / S;     // steps whose slots all exist
    const int64_t steps = (nblk + S - 1) / S;
    double acc[R][NV];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[r][i] = 0.0;
        const int64_t v = threadIdx.x + (int64_t)r * BS;
        // the two doubles of step b
        auto load2 = [&](int64_t b, double (&o)[2]) {
            const double* q = part + 2 * b;
            if constexpr (COHERENT) {
                o[0] = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                o[1] = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const double2 d = *reinterpret_cast<const double2*>(q);
                o[0] = d.x;
                o[1] = d.y;
            }
        };
        auto add2 = [&](const double (&o)[2]) {
            if constexpr (NV == 1) {
                acc[r][0] += o[0];
                acc[r][0] += o[1];
            } else {
                acc[r][0] += o[0];
                acc[r][1] += o[1];
            }
        };
        int64_t b = v;
        // U steps' loads in flight, added in step order: the latency of
        // reading partials written by other XCDs sets the finalize launch's
        // time (32 in flight); inside a main kernel (COHERENT) 8 keep its
        // registers low
        auto chunk = [&](auto U_) {
            constexpr int U = decltype(U_)::value;
            for (; b + (U - 1) * (int64_t)kFinalThreads < full; b += U * (int64_t)kFinalThreads) {
                double t[U][2];
#pragma unroll
                for (int u = 0; u < U; ++u) load2(b + (int64_t)u * kFinalThreads, t[u]);
#pragma unroll
                for (int u = 0; u < U; ++u) add2(t[u]);
            }
        };
        if constexpr (!COHERENT) chunk(std::integral_constant<int, 32>{});
        chunk(std::integral_constant<int, 8>{});
        for (; b < steps; b += kFinalThreads) {
            if (b < full) {
                double t[2];
                load2(b, t);
                add2(t);
            } else {   // the last slot of an odd count (one-value reductions)
                acc[r][0] += COHERENT ? __hip_atomic_load(part + 2 * b, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                      : part[2 * b];
            }
        }
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[r][i] = wave_sum(acc[r][i]);
    }
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int i = 0; i < NV; ++i) sm[wave + r * (BS / kWave)][i] = acc[r][i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double sum = 0.0;
        for (int w = 0; w < kWavesV; ++w) sum += sm[w][i];
        tot[i] = sum;
    }
    __syncthreads();
}

// Publish this workgroup's sums of v in slot blk of part (component i of
// slot b at part[b * NV + i]: the slots of a reduction of one value are
// dense, those of two values one 16-byte pair each).
//   mode 0: the workgroup that finishes last (atomic ticket) totals all slots
//           and returns true with the totals in tot -- the scalar step then
//           runs inside this kernel, at the price of device-scope fences in
//           every workgroup;
//   mode 1: plain stores only; a separate finalize launch totals the slots.
// Both modes add the same numbers in the same order.
template <int NV>
__device__ __forceinline__ bool publish(double (&v)[NV], double* part, int64_t blk, int64_t nblk,
                                        uint32_t* ticket, int mode, double (&tot)[NV])
{
    double bs[NV];
    block_sum<NV>(v, bs);
    if (mode != 0) {
        if (threadIdx.x == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) part[blk * NV + i] = bs[i];
        }
        return false;
    }
    __shared__ int is_last;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            __hip_atomic_store(&part[blk * NV + i], bs[i], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t t = atomicAdd(ticket, 1u);
        is_last = (t == (uint32_t)(nblk - 1));
        __threadfence();
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    sum_partials<NV, true, kBlock>(part, nblk, tot);
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
