// kernels.hip -- the MPPI hot path on gfx950.
//
//   rollout_kernel  (a1-a9): one sample per lane.  Noise from in-register
//                   Philox, the per-step dynamics/cost of dyn.hpp, FP32 (or
//                   FP64) cost accumulation; writes S_k and du[t][j][k]
//                   (k fastest, so a wave's stores are coalesced).
//   weights_kernel  (a10-a12): Eq. 4 with the minimum-cost shift.  Every
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

template <typename R, bool FORCE>
__global__ __launch_bounds__(kRolloutBlock) void rollout_kernel(
    const ModelM<R>* __restrict__ Mp, const CostM<R>* __restrict__ Cp, const double* __restrict__ q0,
    const double* __restrict__ qd0, const double* __restrict__ target, const double* __restrict__ U_nom,
    uint64_t seed, uint32_t tick, int K, int T, R* __restrict__ noise, R* __restrict__ S)
{
    __shared__ R Us[kMaxT * NJ];
    for (int i = threadIdx.x; i < T * NJ; i += blockDim.x) Us[i] = R(U_nom[i]);
    __syncthreads();
    const ModelM<R>& M = *Mp;
    const CostM<R>& C = *Cp;
    TargetM<R> tg;
    make_target(target, tg);
    R q[NJ], qd[NJ], te[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) { q[j] = R(q0[j]); qd[j] = R(qd0[j]); te[j] = R(0); }
    if (C.ext_mode == EXTW_CONST) const_ext_torque(M, C, q, te);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K) {
        R s = rollout_sample<R, FORCE>(M, C, tg, q, qd, te, Us, T, seed, tick, (uint32_t)k,
                                       noise + k, (size_t)K);
        S[k] = finite_(s) ? s : R(INFINITY);
    }
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

template <typename R, bool FORCE> static hipError_t rollout_t(const RolloutArgs& a, hipStream_t s)
{
    dim3 grid((a.K + kRolloutBlock - 1) / kRolloutBlock);
    hipLaunchKernelGGL((rollout_kernel<R, FORCE>), grid, dim3(kRolloutBlock), 0, s,
                       (const ModelM<R>*)a.model, (const CostM<R>*)a.cost, a.q0, a.qd0, a.target,
                       a.U_nom, a.seed, (uint32_t)a.tick, a.K, a.T, (R*)a.noise, (R*)a.costs);
    return hipGetLastError();
}

hipError_t launch_rollout(int precision, bool force, const RolloutArgs& a, hipStream_t s)
{
    if (a.T < 1 || a.T > kMaxT || a.K < 1) return hipErrorInvalidValue;
    if (precision == MPPI_FP64) return force ? rollout_t<double, true>(a, s) : rollout_t<double, false>(a, s);
    return force ? rollout_t<float, true>(a, s) : rollout_t<float, false>(a, s);
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
