// kernels.hip -- the MPPI hot path on gfx950.
//
//   update_kernel   (a1-a12): one sample per lane.  Noise from in-register
//                   Philox, the per-step dynamics/cost of dyn.hpp, FP32 (or
//                   FP64) cost accumulation; writes S_k and du[t][j][k]
//                   (k fastest, so a wave's stores are coalesced); then the
//                   Eq. 4 weighting as per-wave partials merged by the last
//                   block (one launch per update).
//   weights_kernel  (a10-a12 alone, on given costs and noise).  Every
//                   block recomputes S_min and eta = sum_k omega_k over the
//                   K costs (L2-resident) and reduces omega_k du[row][k] for
//                   its rows with wave shuffles; writes U_new and the shifted
//                   warm start.
//   prep_model_kernel: parallel-axis shift of the link inertias (create).
//   plant_kernel:   FP64 zero-order-hold plant for the closed loop.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "launch.hpp"
#include "model_prep.hpp"
#include "rollout.hpp"

namespace mppi {

__global__ void prep_model_kernel(const mppi_robot_params* __restrict__ P, ModelM<float>* __restrict__ Mf,
                                  ModelM<double>* __restrict__ Md)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        prep_model(*P, *Mf);
        prep_model(*P, *Md);
    }
}

template <typename A> __device__ __forceinline__ A wave_min(A v);
template <typename A> __device__ __forceinline__ A wave_sum(A v);

// One MPPI update in one launch (a1-a12).  Each block is one wave of 64
// samples (one per lane).  Every lane rolls out its sample, writes S_k and
// keeps du[t][j] in a padded LDS tile (rows x 65) when it fits, else in the
// global noise buffer (also written when the caller asks for the noise).
// The wave then reduces its samples to a partial of Eq. 4 with its own
// shift m_w = min S_k:
//   s_w = sum_k exp((m_w - S_k)/lambda),  V_w[r] = sum_k exp(...) du_k[r].
// The last block to finish (device-scope counter) merges the partials with
// the log-sum-exp rule m = min m_w, f_w = exp((m - m_w)/lambda),
// U_new[r] = U_nom[r] + sum_w f_w V_w[r] / sum_w f_w s_w, which equals
// Eq. 4b with S_min = m exactly in real arithmetic.  With merge == 0 the
// kernel stops after the rollouts (costs and global noise only).
constexpr int kLdsRowPad = 65;
constexpr int kMaxDynLds = 48 * 1024;

template <typename R, typename A, bool FORCE>
__global__ __launch_bounds__(kRolloutBlock) void update_kernel(
    const ModelM<R>* __restrict__ Mp, const CostM<R>* __restrict__ Cp, const double* __restrict__ q0,
    const double* __restrict__ qd0, const double* __restrict__ target, const double* U_nom,
    uint64_t seed, uint32_t tick, int K, int T, double lambda, R* __restrict__ noise,
    R* __restrict__ S, int merge, int lds_noise, A* __restrict__ parts, unsigned int* __restrict__ counter,
    double* U_new, double* __restrict__ U_shift, int* __restrict__ status)
{
    extern __shared__ char dyn_lds[];
    __shared__ R Us[kMaxT * NJ];
    __shared__ A wl[64];
    __shared__ int last;
    // the model and cost constants are read from LDS (uniform addresses):
    // ~250 values are more than the scalar registers hold across a step
    __shared__ ModelM<R> Msh;
    __shared__ CostM<R> Csh;
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(Mp);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&Msh);
        for (int i = threadIdx.x; i < (int)(sizeof(ModelM<R>) / 4); i += blockDim.x) dst[i] = src[i];
        src = reinterpret_cast<const uint32_t*>(Cp);
        dst = reinterpret_cast<uint32_t*>(&Csh);
        for (int i = threadIdx.x; i < (int)(sizeof(CostM<R>) / 4); i += blockDim.x) dst[i] = src[i];
    }
    for (int i = threadIdx.x; i < T * NJ; i += blockDim.x) Us[i] = R(U_nom[i]);
    __syncthreads();
    const ModelM<R>& M = Msh;
    const CostM<R>& C = Csh;
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    R* tile = reinterpret_cast<R*>(dyn_lds);   // [rows][65] when lds_noise
    R s = R(INFINITY);
    {
        TargetM<R> tg;
        make_target(target, tg);
        R q[NJ], qd[NJ], te[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) { q[j] = R(q0[j]); qd[j] = R(qd0[j]); te[j] = R(0); }
        if (C.ext_mode == EXTW_CONST) const_ext_torque(M, C, q, te);
        if (k < K) {
            R v = rollout_sample<R, FORCE>(M, C, tg, q, qd, te, Us, T, seed, tick, (uint32_t)k,
                                           noise ? noise + k : nullptr, (size_t)K,
                                           lds_noise ? tile + lane : nullptr, kLdsRowPad);
            s = finite_(v) ? v : R(INFINITY);
            S[k] = s;
        } else if (lds_noise) {
            for (int r = 0; r < T * NJ; ++r) tile[r * kLdsRowPad + lane] = R(0);
        }
    }
    if (!merge) return;

    // ---- wave partial
    const int rows = T * NJ;
    const int P = 2 + rows;
    const int kbase = blockIdx.x * blockDim.x;
    const int nk = min(64, K - kbase);
    const A inf = A(INFINITY), il = A(1) / A(lambda);
    A m = wave_min(s < R(INFINITY) ? A(s) : inf);
    A w = (s < R(INFINITY)) ? exp((m - A(s)) * il) : A(0);
    A sw = wave_sum(w);
    wl[lane] = w;
    __syncthreads();
    A* part = parts + (size_t)blockIdx.x * P;
    if (lds_noise) {
        // lane r sums row r of the tile (row stride 65: conflict-free)
        for (int r = lane; r < rows; r += 64) {
            const R* row = tile + r * kLdsRowPad;
            A acc = A(0);
#pragma unroll 16
            for (int i = 0; i < 64; ++i) acc += wl[i] * A(row[i]);
            part[2 + r] = acc;
        }
    } else {
        // global noise: stage 64 rows at a time with coalesced loads along k
        A* trt = reinterpret_cast<A*>(dyn_lds);   // [64][65]
        for (int c0 = 0; c0 < rows; c0 += 64) {
            const int nr = min(64, rows - c0);
#pragma unroll 8
            for (int rr = 0; rr < nr; ++rr)
                trt[rr * kLdsRowPad + lane] = lane < nk ? A(noise[(size_t)(c0 + rr) * K + kbase + lane]) : A(0);
            __syncthreads();
            if (lane < nr) {
                A acc = A(0);
#pragma unroll 16
                for (int i = 0; i < 64; ++i) acc += wl[i] * trt[lane * kLdsRowPad + i];
                part[2 + c0 + lane] = acc;
            }
            __syncthreads();
        }
    }
    if (lane == 0) { part[0] = m; part[1] = sw; }

    // ---- the last block merges all partials
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    const int np = gridDim.x;
    A mg = inf;
    for (int p = lane; p < np; p += 64) mg = fmin(mg, parts[(size_t)p * P]);
    mg = wave_min(mg);
    if (!(mg < inf)) {  // no finite cost: keep the nominal sequence
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
        if (lane == 0) *counter = 0u;
        return;
    }
    A eta = A(0);
    for (int p = lane; p < np; p += 64) {
        A mp = parts[(size_t)p * P];
        if (mp < inf) eta += exp((mg - mp) * il) * parts[(size_t)p * P + 1];
    }
    eta = wave_sum(eta);
    // rows r0 + lane: V[r] = sum_p f_p V_p[r], f_p = exp((m - m_p)/lambda),
    // 64 partials at a time (factors staged in LDS, loads coalesced along r)
    for (int r0 = 0; r0 < rows; r0 += 64) {
        const int r = r0 + lane;
        A acc = A(0);
        for (int p0 = 0; p0 < np; p0 += 64) {
            const int p = p0 + lane;
            A f = A(0);
            if (p < np) {
                A mp = parts[(size_t)p * P];
                f = (mp < inf) ? exp((mg - mp) * il) : A(0);
            }
            __syncthreads();
            wl[lane] = f;
            __syncthreads();
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
    if (lane == 0) *counter = 0u;
}

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

template <typename R, typename A, int ROWS>
__global__ __launch_bounds__(kWeightsBlock) void weights_kernel(
    const R* __restrict__ S, const R* __restrict__ noise, const double* __restrict__ U_nom,
    double* U_new, double* __restrict__ U_shift, int* __restrict__ status, int K, int T, double lambda)
{
    constexpr int NW = kWeightsBlock / 64;
    __shared__ A red[NW][ROWS + 1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int rows = T * NJ, r0 = blockIdx.x * ROWS;
    const A inf = A(INFINITY);

    // S_min over the finite costs (Sec. II: shifted costs S - S_min)
    A m = inf;
    for (int k = tid; k < K; k += kWeightsBlock) {
        A s = A(S[k]);
        if (s - s == A(0)) m = fmin(m, s);
    }
    m = wave_min(m);
    if (lane == 0) red[wid][0] = m;
    __syncthreads();
    m = red[0][0];
#pragma unroll
    for (int w = 1; w < NW; ++w) m = fmin(m, red[w][0]);
    __syncthreads();

    if (!(m < inf)) {  // no finite cost: keep the nominal sequence
        if (tid < ROWS && r0 + tid < rows) {
            const int row = r0 + tid, t = row / NJ, j = row % NJ;
            const double un = U_nom[row];
            U_new[row] = un;
            if (U_shift) {
                if (t >= 1) U_shift[(t - 1) * NJ + j] = un;
                if (t == T - 1) U_shift[t * NJ + j] = un;
            }
        }
        if (status && blockIdx.x == 0 && tid == 0) *status = MPPI_ENONFINITE;
        return;
    }

    // omega_k = exp(-(S_k - S_min)/lambda)  (Eq. 4a); eta and sum omega du (Eq. 4b)
    const A il = A(1) / A(lambda);
    A eta = A(0), acc[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) acc[r] = A(0);
    for (int k = tid; k < K; k += kWeightsBlock) {
        A s = A(S[k]);
        A w = (s - s == A(0)) ? exp((m - s) * il) : A(0);
        eta += w;
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
            if (r0 + r < rows) acc[r] += w * A(noise[(size_t)(r0 + r) * K + k]);
    }
    eta = wave_sum(eta);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) acc[r] = wave_sum(acc[r]);
    if (lane == 0) {
        red[wid][0] = eta;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) red[wid][1 + r] = acc[r];
    }
    __syncthreads();
    if (tid < ROWS && r0 + tid < rows) {
        A e = red[0][0], a = red[0][1 + tid];
#pragma unroll
        for (int w = 1; w < NW; ++w) { e += red[w][0]; a += red[w][1 + tid]; }
        const int row = r0 + tid, t = row / NJ, j = row % NJ;
        const double un = U_nom[row] + double(a / e);
        U_new[row] = un;
        if (U_shift) {
            if (t >= 1) U_shift[(t - 1) * NJ + j] = un;
            if (t == T - 1) U_shift[t * NJ + j] = un;
        }
    }
    if (status && blockIdx.x == 0 && tid == 0) *status = MPPI_OK;
}

__global__ void plant_kernel(const ModelM<double>* __restrict__ Mp, const CostM<double>* __restrict__ Cp,
                             double* q, double* qd, const double* __restrict__ u, double dt, int substeps)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const ModelM<double>& M = *Mp;
    const CostM<double>& C = *Cp;
    double tau[NJ], qq[NJ], qv[NJ];
    for (int j = 0; j < NJ; ++j) {
        double lim = M.L[j].taumax;
        tau[j] = fmin(fmax(u[j], -lim), lim);
        qq[j] = q[j];
        qv[j] = qd[j];
    }
    const int ext = C.ext_mode == EXTW_WALL ? EXTW_WALL : (C.ext_mode == EXTW_CONST ? EXTW_CONST : EXTW_NONE);
    const double h = dt / substeps;
    for (int s = 0; s < substeps; ++s) {
        StepOut<double> o;
        dyn_step<double, false>(M, C, ext, qq, qv, tau, tau, o);
        for (int j = 0; j < NJ; ++j) {
            qv[j] += o.qdd[j] * h;
            qq[j] += qv[j] * h;
        }
    }
    for (int j = 0; j < NJ; ++j) { q[j] = qq[j]; qd[j] = qv[j]; }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_prep_model(const mppi_robot_params* d_raw, ModelM<float>* d_mf, ModelM<double>* d_md,
                             hipStream_t s)
{
    hipLaunchKernelGGL(prep_model_kernel, dim3(1), dim3(64), 0, s, d_raw, d_mf, d_md);
    return hipGetLastError();
}

template <typename R, typename A, bool FORCE> static hipError_t update_t(const UpdateArgs& a, hipStream_t s)
{
    dim3 grid((a.K + kRolloutBlock - 1) / kRolloutBlock);
    const size_t rows = (size_t)a.T * NJ;
    const size_t tile = rows * kLdsRowPad * sizeof(R);
    const int lds_noise = a.merge && tile <= (size_t)kMaxDynLds;
    const size_t dyn = lds_noise ? tile : (a.merge ? 64 * kLdsRowPad * sizeof(A) : 0);
    // global noise: always for rollouts-only launches and the global-tile
    // path; otherwise only when the caller asked for it
    R* noise = (R*)a.noise;
    if (a.merge && lds_noise && !a.want_noise) noise = nullptr;
    hipLaunchKernelGGL((update_kernel<R, A, FORCE>), grid, dim3(kRolloutBlock), dyn, s,
                       (const ModelM<R>*)a.model, (const CostM<R>*)a.cost, a.q0, a.qd0, a.target, a.U_nom,
                       a.seed, (uint32_t)a.tick, a.K, a.T, a.lambda, noise, (R*)a.costs, a.merge, lds_noise,
                       (A*)a.parts, a.counter, a.U_new, a.U_shift, a.status);
    return hipGetLastError();
}

hipError_t launch_update(int precision, bool acc64, bool force, const UpdateArgs& a, hipStream_t s)
{
    if (a.T < 1 || a.T > kMaxT || a.K < 1) return hipErrorInvalidValue;
    if (precision == MPPI_FP64)
        return force ? update_t<double, double, true>(a, s) : update_t<double, double, false>(a, s);
    if (acc64) return force ? update_t<float, double, true>(a, s) : update_t<float, double, false>(a, s);
    return force ? update_t<float, float, true>(a, s) : update_t<float, float, false>(a, s);
}

size_t update_parts_bytes(int K, int T)
{
    return (size_t)((K + kRolloutBlock - 1) / kRolloutBlock) * (2 + (size_t)T * NJ) * sizeof(double);
}

template <typename R, typename A> static hipError_t weights_t(const WeightsArgs& a, hipStream_t s)
{
    dim3 grid((a.T * NJ + kWeightsRows - 1) / kWeightsRows);
    hipLaunchKernelGGL((weights_kernel<R, A, kWeightsRows>), grid, dim3(kWeightsBlock), 0, s,
                       (const R*)a.costs, (const R*)a.noise, a.U_nom, a.U_new, a.U_shift, a.status, a.K,
                       a.T, a.lambda);
    return hipGetLastError();
}

hipError_t launch_weights(int precision, bool acc64, const WeightsArgs& a, hipStream_t s)
{
    if (precision == MPPI_FP64) return weights_t<double, double>(a, s);
    return acc64 ? weights_t<float, double>(a, s) : weights_t<float, float>(a, s);
}

hipError_t launch_plant(const ModelM<double>* M, const CostM<double>* C, double* q, double* qd,
                        const double* u, double dt, int substeps, hipStream_t s)
{
    hipLaunchKernelGGL(plant_kernel, dim3(1), dim3(64), 0, s, M, C, q, qd, u, dt, substeps);
    return hipGetLastError();
}

}  // namespace mppi
