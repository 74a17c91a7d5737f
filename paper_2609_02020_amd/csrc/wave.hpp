// wave.hpp -- wave-level pieces shared by the single-problem and the
// batched update kernels: reductions, the per-wave partial of Eq. 4 and the
// merge of the partials of one problem.
//
// Eq. 4 as partials: a wave of 64 samples with costs S_k reduces to
//   m = min_k S_k,  s = sum_k exp((m - S_k)/lambda),
//   V[r] = sum_k exp((m - S_k)/lambda) du_k[r],   r = 7 t + j.
// Partials (m_w, s_w, V_w) of one problem merge exactly (log-sum-exp rule):
//   m = min_w m_w, f_w = exp((m - m_w)/lambda),
//   U_new[r] = U_nom[r] + sum_w f_w V_w[r] / sum_w f_w s_w,
// which is Eq. 4b with S_min = m (Sec. II: the shift leaves the result
// unchanged).  Non-finite costs weigh zero; a problem with no finite cost
// keeps its nominal sequence and reports MPPI_ENONFINITE.
#pragma once

#include <hip/hip_runtime.h>

#include "mppi.h"
#include "rollout.hpp"

namespace mppi {

constexpr int kLdsRowPad = 65;   // row stride of the [rows][64] transpose tiles

template <typename A> __device__ __forceinline__ A wave_min(A v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
template <typename A> __device__ __forceinline__ A wave_sum(A v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
// orders the LDS accesses of one wave (cross-lane exchange through LDS)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// copies `bytes` (a multiple of 4) from global memory to LDS with one wave
// Copies an object of T by the 64 lanes of a wave, every load issued before
// the first store (one memory round trip, where a loop of load-store pairs
// waits for each load in turn).
template <typename T> __device__ __forceinline__ void wave_copy(T* dst, const T* src, int lane)
{
    static_assert(sizeof(T) % 4 == 0, "copied as 32-bit words");
    constexpr int W = sizeof(T) / 4, N = (W + 63) / 64;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    uint32_t v[N];
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = (lane + 64 * n < W) ? s[lane + 64 * n] : 0u;
#pragma unroll
    for (int n = 0; n < N; ++n)
        if (lane + 64 * n < W) d[lane + 64 * n] = v[n];
}

// Per-wave partial.  s_lane: this lane's cost (+inf if invalid or
// non-finite).  Noise source: `tile` (LDS, [rows][kLdsRowPad], column =
// lane) if non-null, otherwise regenerated from the Philox counters of
// (seed, tick, k, t) with sigma from C (bitwise the rollout's noise).  tr: LDS
// scratch [64][kLdsRowPad] of R; wl: LDS scratch [64] of A.  part: global
// [2 + rows].  Invalid lanes must pass s_lane = +inf (weight 0).
template <typename R, typename A>
__device__ void wave_partial(R s_lane, int lane, int T, double lambda, const R* tile, const CostM<R>& C,
                             uint64_t seed, uint32_t tick, uint32_t k, R* tr, A* wl, A* part)
{
    const int rows = T * NJ;
    const A inf = A(INFINITY), il = A(1) / A(lambda);
    const bool fin = s_lane < R(INFINITY);
    const A m = wave_min(fin ? A(s_lane) : inf);
    const A w = fin ? exp((m - A(s_lane)) * il) : A(0);
    const A sw = wave_sum(w);
    wl[lane] = w;
    wave_sync();
    if (tile) {
        for (int r = lane; r < rows; r += 64) {
            const R* row = tile + r * kLdsRowPad;
            A acc = A(0);
#pragma unroll 16
            for (int i = 0; i < 64; ++i) acc += wl[i] * A(row[i]);
            part[2 + r] = acc;
        }
    } else {
        // 9 steps (63 rows) at a time: lane stages du[t][j] in column `lane`,
        // then lane r sums w_i du_i over row r; du carries the time
        // recursion of correlated noise across the blocks
        R du[NJ];
        for (int t0 = 0; t0 < T; t0 += 9) {
            const int nt = min(9, T - t0);
            for (int tt = 0; tt < nt; ++tt) {
                R z[8];
                normals8<R>(seed, tick, k, (uint32_t)(t0 + tt), z);
                noise_step(C, z, du, t0 + tt);
#pragma unroll
                for (int j = 0; j < NJ; ++j) tr[(tt * NJ + j) * kLdsRowPad + lane] = du[j];
            }
            wave_sync();
            const int nr = nt * NJ;
            if (lane < nr) {
                A acc = A(0);
#pragma unroll 16
                for (int i = 0; i < 64; ++i) acc += wl[i] * A(tr[lane * kLdsRowPad + i]);
                part[2 + t0 * NJ + lane] = acc;
            }
            wave_sync();
        }
    }
    if (lane == 0) { part[0] = m; part[1] = sw; }
}

// Merge of np partials [np][2 + rows] of one problem by one wave; writes
// U_new, U_shift (may be null) and *status (may be null).  wl: LDS [64] of A.
template <typename A>
__device__ void wave_merge(const A* parts, int np, int T, double lambda, const double* U_nom, double* U_new,
                           double* U_shift, int* status, int lane, A* wl)
{
    const int rows = T * NJ, P = 2 + rows;
    const A inf = A(INFINITY), il = A(1) / A(lambda);
    A mg = inf;
    for (int p = lane; p < np; p += 64) mg = fmin(mg, parts[(size_t)p * P]);
    mg = wave_min(mg);
    if (!(mg < inf)) {
        for (int r = lane; r < rows; r += 64) {
            const int t = r / NJ, j = r % NJ;
            const double un = U_nom[r];
            U_new[r] = un;
            if (U_shift) {
                if (t >= 1) U_shift[(t - 1) * NJ + j] = un;
                if (t == T - 1) U_shift[t * NJ + j] = un;
            }
        }
        if (status && lane == 0) *status = MPPI_ENONFINITE;
        return;
    }
    A eta = A(0);
    for (int p = lane; p < np; p += 64) {
        const A mp = parts[(size_t)p * P];
        if (mp < inf) eta += exp((mg - mp) * il) * parts[(size_t)p * P + 1];
    }
    eta = wave_sum(eta);
    for (int r0 = 0; r0 < rows; r0 += 64) {
        const int r = r0 + lane;
        A acc = A(0);
        for (int p0 = 0; p0 < np; p0 += 64) {
            const int p = p0 + lane;
            A f = A(0);
            if (p < np) {
                const A mp = parts[(size_t)p * P];
                f = (mp < inf) ? exp((mg - mp) * il) : A(0);
            }
            wave_sync();
            wl[lane] = f;
            wave_sync();
            if (r < rows) {
                if (np - p0 >= 64) {
                    A v[64];
#pragma unroll
                    for (int i = 0; i < 64; ++i) v[i] = parts[(size_t)(p0 + i) * P + 2 + r];
#pragma unroll
                    for (int i = 0; i < 64; ++i) acc += wl[i] * v[i];
                } else {
                    for (int i = 0; i < np - p0; ++i) acc += wl[i] * parts[(size_t)(p0 + i) * P + 2 + r];
                }
            }
        }
        if (r < rows) {
            const int t = r / NJ, j = r % NJ;
            const double un = U_nom[r] + double(acc / eta);
            U_new[r] = un;
            if (U_shift) {
                if (t >= 1) U_shift[(t - 1) * NJ + j] = un;
                if (t == T - 1) U_shift[t * NJ + j] = un;
            }
        }
    }
    if (status && lane == 0) *status = MPPI_OK;
}

}  // namespace mppi
