// kernels.hip -- the MPPI hot path on gfx950.
//
//   update_group_kernel + group_merge_kernel (a1-a12, the default for FP32
//                   rollouts): eight lanes per sample (group.hpp) on
//                   dynamics/cost wave pairs, workgroup partials of Eq. 4,
//                   merged by a second launch.
//   update_split_kernel (two waves per 64 samples) and
//   update_kernel   (a1-a12): one sample per lane.  Noise from in-register
//                   Philox, the per-step dynamics/cost of dyn.hpp, FP32 (or
//                   FP64) cost accumulation; writes S_k and du[t][j][k]
//                   (k fastest, so a wave's stores are coalesced); then the
//                   Eq. 4 weighting as per-wave partials merged by the last
//                   block (one launch per update).
//   batch_kernel    (a13): one persistent launch over the 64-sample tiles of
//                   many problems, one sample per lane.
//   weights_kernel  (a10-a12 alone, on given costs and noise).  Every
//                   block recomputes S_min and eta = sum_k omega_k over the
//                   K costs (L2-resident) and reduces omega_k du[row][k] for
//                   its rows with wave shuffles; writes U_new and the shifted
//                   warm start.
//   prep_model_kernel: parallel-axis shift of the link inertias (create).
//   plant_kernel, batch_plant_kernel: FP64 zero-order-hold plant for the
//                   closed loop (one problem, or one workgroup per problem).
//   select_kernel, batch_select_kernel: noise-free costs of the warm start
//                   and a proposed nominal sequence; keeps the cheaper.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>

#include "launch.hpp"
#include "model_prep.hpp"
#include "rollout.hpp"
#include "wave.hpp"
#include "group.hpp"

namespace mppi {

__global__ void prep_model_kernel(const mppi_robot_params* __restrict__ P, ModelM<float>* __restrict__ Mf,
                                  ModelM<double>* __restrict__ Md)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        prep_model(*P, *Mf);
        prep_model(*P, *Md);
    }
}

// One MPPI update in one launch (a1-a12).  Each workgroup is one wave of
// 64 samples (one per lane).  Every lane rolls out its sample and writes
// S_k; the noise goes to a padded LDS tile when it fits (else it is
// regenerated from the Philox counters for the weighting) and to the
// global noise buffer only when the caller asks for it.  The wave reduces
// its samples to a partial of Eq. 4 (wave.hpp) and the last workgroup to
// finish merges the partials.  With merge == 0 the kernel stops after the
// rollouts (costs and global noise only).
constexpr int kMaxDynLds = 48 * 1024;

template <typename R, typename A, bool FORCE, bool EXPLICIT, bool COLL>
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
    // Model constants (~190 values) are read through the scalar cache at
    // uniform addresses, re-issued every step (rollout.hpp per_step), so
    // their scalar-register lifetimes stay within a step; the cost
    // constants are read from an LDS copy, which measured faster than
    // adding them to the scalar stream.
    __shared__ CostM<R> Csh;
    const int lane = threadIdx.x & 63;
    wave_copy(&Csh, Cp, lane);
    for (int i = threadIdx.x; i < T * NJ; i += blockDim.x) Us[i] = R(U_nom[i]);
    __syncthreads();
    const ModelM<R>& M = *Mp;
    const CostM<R>& C = Csh;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    R* tile = reinterpret_cast<R*>(dyn_lds);   // [rows][65] (noise) or [64][65] (regeneration)
    R s = R(INFINITY);
    {
        TargetM<R> tg;
        make_target(target, tg);
        R q[NJ], qd[NJ], te[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) { q[j] = R(q0[j]); qd[j] = R(qd0[j]); te[j] = R(0); }
        if (C.ext_mode == EXTW_CONST) const_ext_torque(M, C, q, te);
        if (k < K) {
            R v = rollout_sample<R, FORCE, EXPLICIT, COLL>(M, C, tg, q, qd, te, Us, T, seed, tick, (uint32_t)k,
                                           noise ? noise + k : nullptr, (size_t)K,
                                           lds_noise ? tile + lane : nullptr, kLdsRowPad);
            s = finite_(v) ? v : R(INFINITY);
            S[k] = s;
        } else if (lds_noise) {
            for (int r = 0; r < T * NJ; ++r) tile[r * kLdsRowPad + lane] = R(0);
        }
    }
    if (!merge) return;

    const int P = 2 + T * NJ;
    wave_sync();
    wave_partial<R, A>(s, lane, T, lambda, lds_noise ? tile : nullptr, C, seed, tick, (uint32_t)k, tile, wl,
                       parts + (size_t)blockIdx.x * P);

    // the last workgroup merges all partials
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    wave_merge<A>(parts, gridDim.x, T, lambda, U_nom, U_new, U_shift, status, lane, wl);
    if (lane == 0) *counter = 0u;
}

// The same update with two waves per 64 samples (FP32, articulated-body
// dynamics): wave 0 runs the dynamics of every step (the sequential chain
// of a sample), wave 1 draws the perturbations one step ahead and evaluates
// the force estimate of Eq. 13 (FORCE) and the running cost one step
// behind, from what wave 0 leaves in LDS.  With 64 waves for K = 4096
// the single-wave update is bound by one wave's instruction stream per
// SIMD; the split halves that stream's length on the critical path and
// puts a second SIMD of each CU to work.  Per sample the arithmetic is the
// single-wave update's (the same functions in the same order).
//
// Per step s (both waves meet at one barrier per step):
//   wave 0: du_s from nb[s&1] -> v, tau; dyn_step (factors into hb[s&1]); Euler
//   wave 1: noise of step s+1 -> nb[(s+1)&1]; step s-1 from hb[(s-1)&1]:
//           F_ee (FORCE), l(x, v), S += l
// The handoff is struct-of-arrays in LDS, [value][lane] (conflict-free): the flat ForceIn
// (stored by dyn_step link by link, as soon as the step is done with each
// value) followed by the pre-step q, qd, the sampled v and the EE pose.
// The zero-velocity solve of the force estimate runs on wave 1 too.
constexpr int kHoQ = kFiCount, kHoQd = kHoQ + NJ, kHoV = kHoQd + NJ, kHoPee = kHoV + NJ, kHoRn = kHoPee + 3,
              kHandoff = kHoRn + 9;   // 127 values per sample

template <bool FORCE>
__device__ __forceinline__ void handoff_read(const float* h, ForceIn<float>& fi, float* q, float* qd, float* v,
                                             float* pee, float* Rn)
{
    if constexpr (FORCE) {
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                fi.z[i][c] = h[(kFiZ + 3 * i + c) * 64];
                fi.rr[i][c] = h[(kFiRr + 3 * i + c) * 64];
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) fi.U[i][c] = h[(kFiU + 6 * i + c) * 64];
            fi.iD[i] = h[(kFiD + i) * 64];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) fi.ree[c] = h[(kFiRee + c) * 64];
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) { q[j] = h[(kHoQ + j) * 64]; qd[j] = h[(kHoQd + j) * 64]; v[j] = h[(kHoV + j) * 64]; }
#pragma unroll
    for (int c = 0; c < 3; ++c) pee[c] = h[(kHoPee + c) * 64];
#pragma unroll
    for (int c = 0; c < 9; ++c) Rn[c] = h[(kHoRn + c) * 64];
}

template <typename A, bool FORCE, bool COLL>
__global__ __launch_bounds__(128) void update_split_kernel(
    const ModelM<float>* __restrict__ Mp, const CostM<float>* __restrict__ Cp, const double* __restrict__ q0,
    const double* __restrict__ qd0, const double* __restrict__ target, const double* U_nom,
    uint64_t seed, uint32_t tick, int K, int T, double lambda, float* __restrict__ noise,
    float* __restrict__ S, int merge, int lds_noise, A* __restrict__ parts, unsigned int* __restrict__ counter,
    double* U_new, double* __restrict__ U_shift, int* __restrict__ status)
{
    extern __shared__ char dyn_lds[];
    __shared__ float hb[2][kHandoff * 64];
    __shared__ float nb[2][NJ * 64];
    __shared__ float Us[kMaxT * NJ];
    __shared__ A wl[64];
    __shared__ int last;
    __shared__ CostM<float> Csh;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave == 0) wave_copy(&Csh, Cp, lane);
    for (int i = threadIdx.x; i < T * NJ; i += blockDim.x) Us[i] = float(U_nom[i]);
    const int k = blockIdx.x * 64 + lane;
    float* tile = reinterpret_cast<float*>(dyn_lds);   // [rows][65] (noise) or [64][65] (regeneration)
    float* noise_k = (noise && k < K) ? noise + k : nullptr;
    float* tile_k = lds_noise ? tile + lane : nullptr;
    const ModelM<float>& Mc = *Mp;
    const CostM<float>& Cc = Csh;
    __syncthreads();

    float q[NJ], qd[NJ], te[NJ];   // wave 0: the trajectory
    float du[NJ], Ssum = 0.0f;     // wave 1: the noise recursion and the cost
    TargetM<float> tg;
    if (wave == 0) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) { q[j] = float(q0[j]); qd[j] = float(qd0[j]); te[j] = 0.0f; }
        if (Cc.ext_mode == EXTW_CONST) const_ext_torque(Mc, Cc, q, te);
    } else {
        make_target(target, tg);
#pragma unroll
        for (int j = 0; j < NJ; ++j) du[j] = 0.0f;
        float z[8];
        normals8<float>(seed, tick, (uint32_t)k, 0u, z);
        noise_step(Cc, z, du, 0);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            nb[0][j * 64 + lane] = du[j];
            if (noise_k) noise_k[(size_t)j * K] = du[j];
            if (tile_k) tile_k[j * kLdsRowPad] = du[j];
        }
    }
    __syncthreads();
    const int ext = Cc.ext_mode == EXTW_WALL ? EXTW_WALL : EXTW_NONE;
    for (int s = 0; s <= T; ++s) {
        if (wave == 0) {
            if (s < T) {
                const ModelM<float>& M = *per_step(&Mc);
                const CostM<float>& C = *per_step(&Cc);
                float v[NJ], tau[NJ];
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    v[j] = Us[s * NJ + j] + nb[s & 1][j * 64 + lane];
                    tau[j] = v[j] + te[j];
                }
                StepOut<float> o;
                float* h = &hb[s & 1][lane];
                dyn_step<float, FORCE>(M, C, ext, q, qd, tau, v, o, h, 64);
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    h[(kHoQ + j) * 64] = q[j];
                    h[(kHoQd + j) * 64] = qd[j];
                    h[(kHoV + j) * 64] = v[j];
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) h[(kHoPee + c) * 64] = o.pee[c];
#pragma unroll
                for (int c = 0; c < 9; ++c) h[(kHoRn + c) * 64] = o.Rn[c];
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    qd[j] += o.qdd[j] * C.dt;
                    q[j] += qd[j] * C.dt;
                }
            }
        } else {
            const ModelM<float>& M = *per_step(&Mc);
            const CostM<float>& C = *per_step(&Cc);
            if (s + 1 < T) {
                float z[8];
                normals8<float>(seed, tick, (uint32_t)k, (uint32_t)(s + 1), z);
                noise_step(C, z, du, s + 1);
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    nb[(s + 1) & 1][j * 64 + lane] = du[j];
                    if (noise_k) noise_k[(size_t)((s + 1) * NJ + j) * K] = du[j];
                    if (tile_k) tile_k[((s + 1) * NJ + j) * kLdsRowPad] = du[j];
                }
            }
            if (s >= 1) {
                ForceIn<float> fi;
                float qs[NJ], qds[NJ], v[NJ], pee[3], Rn[9];
                handoff_read<FORCE>(&hb[(s - 1) & 1][lane], fi, qs, qds, v, pee, Rn);
                float l = motion_cost(M, C, tg, pee, Rn) + joint_cost(M, C, qs, qds) + torque_cost(M, C, v);
                if constexpr (FORCE) {
                    float F[6];
                    force_estimate(fi, v, M.g, C.force_mode, F);
                    l += force_cost(C, tg, F);
                }
                if constexpr (COLL) l += collision_cost(M, C, qs);
                Ssum += l;
            }
        }
        __syncthreads();
    }
    // terminal cost phi(x_T): wave 0 hands over the final state
    if (wave == 0) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) { nb[0][j * 64 + lane] = q[j]; nb[1][j * 64 + lane] = qd[j]; }
    }
    __syncthreads();
    float s_lane = INFINITY;
    if (wave == 1) {
        float qT[NJ], qdT[NJ], pee[3], Rn[9];
#pragma unroll
        for (int j = 0; j < NJ; ++j) { qT[j] = nb[0][j * 64 + lane]; qdT[j] = nb[1][j * 64 + lane]; }
        fk_ee(Mc, qT, pee, Rn, (float*)nullptr, (float*)nullptr);
        Ssum += Cc.w_T * (motion_cost(Mc, Cc, tg, pee, Rn) + joint_cost(Mc, Cc, qT, qdT));
        if (k < K) {
            s_lane = finite_(Ssum) ? Ssum : INFINITY;
            S[k] = s_lane;
        }
    }
    if (!merge) return;

    const int P = 2 + T * NJ;
    if (wave == 1) {
        wave_sync();
        wave_partial<float, A>(s_lane, lane, T, lambda, lds_noise ? tile : nullptr, Cc, seed, tick, (uint32_t)k,
                               tile, wl, parts + (size_t)blockIdx.x * P);
        __threadfence();
        if (lane == 0) last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || wave == 0) return;
    __threadfence();
    wave_merge<A>(parts, gridDim.x, T, lambda, U_nom, U_new, U_shift, status, lane, wl);
    if (lane == 0) *counter = 0u;
}

// One MPPI update with eight lanes per sample (group.hpp): lane j of a
// group holds joint j, lane 7 the EE frame, and every group of samples is
// served by two waves: a dynamics wave (kinematics, inertias, the rows of M,
// the LDL^T solve of Eq. 6 and the Euler step: the sequential chain of a
// sample) and a cost wave, which draws the perturbations one step ahead and
// evaluates the force estimate of Eq. 13 and the running cost one step
// behind from what the dynamics wave leaves in LDS, the LDL^T factor of M
// included (double-buffered group areas, one barrier per step); in the
// last step, while the cost wave
// evaluates step T - 1, the dynamics wave evaluates the terminal cost of
// x_T.  A workgroup holds kGroupPairs such pairs
// (8 kGroupPairs samples, one wave per SIMD); K = 4096 gives 1024 waves.
// After the horizon the workgroup forms its Eq. 4 partial (wave.hpp
// convention) from the du tile in LDS (or from regenerated noise when the
// tile does not fit); group_merge_kernel, launched next, merges them.  Every
// group runs through the rollout (samples past K too, storing nothing), so
// the DPP moves always see a converged wave.
constexpr int kGroupPairs = 2;
constexpr int kGroupSamples = 8 * kGroupPairs;
constexpr int kGroupThreads = 128 * kGroupPairs;
constexpr int kGroupSteps = 32;   // steps per chunk of the partial's row sums (regenerated noise)
constexpr int kGroupTile = kGroupSamples + 1;   // row stride of the workgroup's du tile

// Lane layout of a wave's eight groups: a row of 16 lanes holds two
// samples interleaved, joint j of sample s in lane 2 j + (s & 1) + 16 (s >> 1),
// so that a row shift by 2 D lanes moves every joint's value D joints along
// its own sample, and lanes with no source (the first or last D joints) read
// 0 from the shift itself.
__device__ __forceinline__ int group_joint(int lane) { return (lane >> 1) & 7; }
__device__ __forceinline__ int group_sample(int lane) { return (lane & 1) | ((lane >> 4) << 1); }

struct DevGroup {
    int j;
    float* shm;
    // joint j - D's value (0 for j < D)
    template <int D> __device__ float shr(float x) const
    {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x110 + 2 * D, 0xF, 0xF, true));
    }
    // joint j - D's value (1 for j < D: the shift leaves the old value)
    template <int D> __device__ float shr_one(float x) const
    {
        return __int_as_float(
            __builtin_amdgcn_update_dpp(__float_as_int(1.0f), __float_as_int(x), 0x110 + 2 * D, 0xF, 0xF, false));
    }
    // x plus joint j - D's value (j < D: plus 0), one DPP add
    template <int D> __device__ float add_shr(float x) const { return x + shr<D>(x); }
    // x plus joint j + D's value (j + D > 7: plus 0), one DPP add
    template <int D> __device__ float add_shl(float x) const
    {
        return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x100 + 2 * D, 0xF, 0xF, true));
    }
    // joint K's value: within every bank of four lanes (joints 2 m, 2 m + 1
    // of both samples) the lanes of joint 2 m + (K & 1) spread over the
    // bank, then bank K / 2 is copied into the other three by two masked
    // row shifts
    template <int K> __device__ float bcast(float x) const
    {
        constexpr int h = 2 * (K & 1);
        int t = __builtin_amdgcn_mov_dpp(__float_as_int(x), h | ((h + 1) << 2) | (h << 4) | ((h + 1) << 6), 0xF, 0xF,
                                         true);
        constexpr int b = K >> 1;
        if (b == 0) {
            t = __builtin_amdgcn_update_dpp(t, t, 0x114, 0xF, 0x2, false);   // bank 1 <- 0
            t = __builtin_amdgcn_update_dpp(t, t, 0x118, 0xF, 0xC, false);   // banks 2, 3 <- 0, 1
        } else if (b == 1) {
            t = __builtin_amdgcn_update_dpp(t, t, 0x104, 0xF, 0x1, false);   // bank 0 <- 1
            t = __builtin_amdgcn_update_dpp(t, t, 0x118, 0xF, 0xC, false);   // banks 2, 3 <- 0, 1
        } else if (b == 2) {
            t = __builtin_amdgcn_update_dpp(t, t, 0x114, 0xF, 0x8, false);   // bank 3 <- 2
            t = __builtin_amdgcn_update_dpp(t, t, 0x108, 0xF, 0x3, false);   // banks 0, 1 <- 2, 3
        } else {
            t = __builtin_amdgcn_update_dpp(t, t, 0x104, 0xF, 0x4, false);   // bank 2 <- 3
            t = __builtin_amdgcn_update_dpp(t, t, 0x108, 0xF, 0x3, false);   // banks 0, 1 <- 2, 3
        }
        return __int_as_float(t);
    }
    // over the group: joints j ^ 1, ^ 2, ^ 4 are lanes ^ 2, ^ 4, ^ 8, each
    // reached by DPP within the row (a quad permutation, then pairs of
    // bank-masked row shifts by 4 and by 8)
    __device__ float sum(float x) const
    {
        x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, true));   // [2,3,0,1]
        int t = __builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x104, 0xF, 0x5, false);   // banks 0, 2 <- +4
        t = __builtin_amdgcn_update_dpp(t, __float_as_int(x), 0x114, 0xF, 0xA, false);       // banks 1, 3 <- -4
        x += __int_as_float(t);
        t = __builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x108, 0xF, 0x3, false);       // banks 0, 1 <- +8
        t = __builtin_amdgcn_update_dpp(t, __float_as_int(x), 0x118, 0xF, 0xC, false);       // banks 2, 3 <- -8
        return x + __int_as_float(t);
    }
    __device__ void sync() const { wave_sync(); }
};

template <typename A, bool FORCE, bool COLL>
__global__ __launch_bounds__(kGroupThreads) void update_group_kernel(
    const ModelM<float>* __restrict__ Mp, const CostM<float>* __restrict__ Cp, const double* __restrict__ q0,
    const double* __restrict__ qd0, const double* __restrict__ target, const double* U_nom,
    uint64_t seed, uint32_t tick, int K, int T, double lambda, float* __restrict__ noise,
    float* __restrict__ S, int merge, int lds_noise, A* __restrict__ parts)
{
    extern __shared__ char dyn_lds[];   // lds_noise: du tile [7T][kGroupTile]
    __shared__ float gx[2][kGroupSamples][kGxCount];
    __shared__ float nb[2][kGroupSamples][8];
    __shared__ float Us[kMaxT * NJ];
    __shared__ CostM<float> Csh;
    __shared__ float sS[kGroupSamples];
    __shared__ A vs[kGroupPairs][kGroupSteps * 8];
    __shared__ A wsm[kGroupSamples];
    __shared__ float tS[kGroupSamples][8];   // the terminal cost's lane shares
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool dyn = wave < kGroupPairs;   // waves 0.. P-1: dynamics, P.. 2P-1: cost
    const int pw = dyn ? wave : wave - kGroupPairs;
    const int j = group_joint(lane), grp = pw * 8 + group_sample(lane), jc = j < NJ ? j : NJ - 1;
    const int k = blockIdx.x * kGroupSamples + grp;
    const bool valid = k < K;
    // set-up from global memory (the cost constants from Cp directly, so that
    // every load is issued before the first barrier)
    const ModelM<float>& M = *Mp;
    GroupLink<float> L;
    group_link(M, *Cp, j, L);
    const float grav[3] = {M.g[0], M.g[1], M.g[2]};
    TargetM<float> tg;
    make_target(target, tg);   // the cost wave's running cost, the dynamics wave's terminal cost
    float q = 0.0f, qd = 0.0f, te = 0.0f;
    if (dyn) {
        float qa[NJ], qda[NJ], tea[NJ];
#pragma unroll
        for (int i = 0; i < NJ; ++i) { qa[i] = float(q0[i]); qda[i] = float(qd0[i]); tea[i] = 0.0f; }
        if (Cp->ext_mode == EXTW_CONST) const_ext_torque(M, *Cp, qa, tea);
#pragma unroll
        for (int i = 0; i < NJ; ++i)
            if (i == j) { q = qa[i]; qd = qda[i]; te = tea[i]; }
    }
    if (wave == 0) wave_copy(&Csh, Cp, lane);
    for (int i = tid; i < T * NJ; i += blockDim.x) Us[i] = float(U_nom[i]);
    const CostM<float>& C = Csh;
    float* tile = reinterpret_cast<float*>(dyn_lds);
    float* nz_out = (valid && noise && j < NJ) ? noise + k : nullptr;
    float* nz_lds = (lds_noise && j < NJ) ? tile + grp : nullptr;
    const int ext = Cp->ext_mode == EXTW_WALL ? EXTW_WALL : EXTW_NONE;

    // the cost wave draws du of step t; du carries the AR(1) recursion
    float du = 0.0f, Sl = 0.0f;
    auto draw = [&](int t) {
        du = group_noise_step(C, L, group_normal<float>(seed, tick, (uint32_t)k, (uint32_t)t, j), du, t);
        nb[t & 1][grp][j] = du;
        if (nz_out) nz_out[(size_t)(t * NJ + j) * K] = du;
        if (nz_lds) nz_lds[(t * NJ + j) * kGroupTile] = du;
    };
    // step 0's draw needs only this lane's sigma (not the LDS cost copy)
    if (!dyn) draw(0);
    const float dt = Cp->dt;   // in a register: the step's last operation reads it
    __syncthreads();
    for (int s = 0; s <= T; ++s) {
        if (dyn) {
            if (s < T) {
                float* X = gx[s & 1][grp];
                const DevGroup g{j, X};
                const float v = (Us[s * NJ + jc] + nb[s & 1][grp][j]) * L.live;
                float p[3], Q[9];
                const float qdd = group_dynamics<float, FORCE, DevGroup, COLL, true>(g, L, C, grav, ext, q, qd, v + te, v, X,
                                                                               nullptr, p, Q);
                qd += qdd * dt;
                q += qd * dt;
            } else {
                // phi(x_T) (lane 7: q = qd = 0), while the cost wave
                // evaluates step T - 1
                const DevGroup g{j, gx[s & 1][grp]};
                tS[grp][j] = group_terminal(g, L, C, tg, q, qd);
            }
        } else {
            if (s + 1 < T) draw(s + 1);
            if (s >= 1) {
                float* X = gx[(s - 1) & 1][grp];
                const DevGroup g{j, X};
                const float* h = X + kGxH + j * 12;
                float pe[3], Re[9];
#pragma unroll
                for (int a = 0; a < 3; ++a) pe[a] = h[a];
#pragma unroll
                for (int a = 0; a < 9; ++a) Re[a] = h[3 + a];
                Sl += group_cost<float, FORCE, COLL, DevGroup, COLL, true>(g, L, C, tg, grav, X, nullptr, h[0], h[1], h[2], pe,
                                                                     Re);
            }
        }
        __syncthreads();
    }
    // the terminal cost from the dynamics wave (ordered by the last barrier)
    if (!dyn) {
        const DevGroup g{j, gx[T & 1][grp]};
        Sl += tS[grp][j];
        const float tot = g.sum(Sl);
        float sv = INFINITY;
        if (valid) {
            sv = finite_(tot) ? tot : INFINITY;
            if (j == 0) S[k] = sv;
        }
        if (j == 0) sS[grp] = sv;
    }
    if (!merge) return;
    __syncthreads();

    // ---- this workgroup's partial of Eq. 4: m, sum of weights, V[7T]
    const A inf = A(INFINITY), il = A(1) / A(lambda);
    A m = inf;
#pragma unroll
    for (int i = 0; i < kGroupSamples; ++i) m = fmin(m, sS[i] < INFINITY ? A(sS[i]) : inf);
    if (tid < kGroupSamples) wsm[tid] = sS[tid] < INFINITY ? exp((m - A(sS[tid])) * il) : A(0);
    __syncthreads();
    // partials: (m, s) of every workgroup in [nb][2], then V in [nb][7T]
    A* part_ms = parts + (size_t)blockIdx.x * 2;
    A* part = parts + (size_t)gridDim.x * 2 + (size_t)blockIdx.x * (T * NJ);
    if (lds_noise) {
        for (int r = tid; r < T * NJ; r += blockDim.x) {
            const float* row = tile + r * kGroupTile;
            A acc = A(0);
#pragma unroll
            for (int i = 0; i < kGroupSamples; ++i) acc += wsm[i] * A(row[i]);
            part[r] = acc;
        }
    } else {
        // regenerated noise: the cost waves' lanes reduce w du over their
        // wave's 8 samples of each joint, then the pairs are summed
        const A wgt = wsm[grp];
        float dr = 0.0f;
        for (int t0 = 0; t0 < T; t0 += kGroupSteps) {
            const int nt = min(kGroupSteps, T - t0);
            if (!dyn) {
                for (int tt = 0; tt < nt; ++tt) {
                    const int t = t0 + tt;
                    dr = group_noise_step(C, L, group_normal<float>(seed, tick, (uint32_t)k, (uint32_t)t, j), dr, t);
                    // over the wave's 8 samples (lane bits 0, 4, 5)
                    A x = wgt * A(dr);
                    x += __shfl_xor(x, 1);
                    x += __shfl_xor(x, 16);
                    x += __shfl_xor(x, 32);
                    if ((lane & 0x31) == 0) vs[pw][tt * 8 + j] = x;
                }
            }
            __syncthreads();
            for (int r = tid; r < nt * NJ; r += blockDim.x) {
                const int tt = r / NJ, jj = r % NJ;
                A acc = A(0);
#pragma unroll
                for (int w = 0; w < kGroupPairs; ++w) acc += vs[w][tt * 8 + jj];
                part[(t0 + tt) * NJ + jj] = acc;
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        A st = A(0);
#pragma unroll
        for (int i = 0; i < kGroupSamples; ++i) st += wsm[i];
        part_ms[0] = m;
        part_ms[1] = st;
    }

    // the partials are merged by group_merge_kernel, launched next on the
    // same stream: the kernel boundary orders them, with no per-workgroup
    // fence (an agent-scope release writes back the XCD's L2, and hundreds
    // of them cost more than the merge)
}

// Eq. 4 from the np workgroup partials of update_group_kernel ((m, s) pairs
// [np][2], then the row sums [np][7T]): workgroup b writes rows
// [kMergeRows b, kMergeRows (b + 1)) of U_new.  Thread (slice, row) takes
// the partials slice, slice + kMergeSlices, ... in batches whose loads are
// issued together (one memory round trip per batch, with this row of U_nom
// in the same trip); a batch is reduced against its own minimum (all its
// exponentials independent) and folded into the running (m, s, V) by the
// log-sum-exp rule of wave.hpp (a new minimum rescales what it has).  The
// slices of a row are then combined through LDS the same way: their minimum
// first, then the rescaled sums.  Every row's slices cover all partials, so
// each row has the full normaliser.  Empty entries (a non-finite minimum,
// or a slot past np, which reads partial 0) enter every step with weight
// zero rather than through a branch: a branch lets the compiler defer the
// loads of such entries past the first wait.
// e^x for the merge's shifted exponents (x <= 0): in FP32 the hardware
// base-2 exponential of x log2(e) (about 1 ulp, plus |x| ulp from the
// scaling, which only the negligible weights reach), libm in FP64
__device__ __forceinline__ float merge_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504f); }
__device__ __forceinline__ double merge_exp(double x) { return exp(x); }
constexpr int kMergeRows = 16;
constexpr int kMergeSlices = kGroupThreads / kMergeRows;
template <typename A>
__global__ __launch_bounds__(kGroupThreads) void group_merge_kernel(const A* __restrict__ parts, int np, int T,
                                                                    double lambda, const double* U_nom,
                                                                    double* U_new, double* __restrict__ U_shift,
                                                                    int* __restrict__ status)
{
    __shared__ A shm[kGroupThreads], shs[kGroupThreads], shv[kGroupThreads];
    const int tid = threadIdx.x, rl = tid % kMergeRows, sl = tid / kMergeRows;
    const int rows = T * NJ;
    const int r = blockIdx.x * kMergeRows + rl;
    const bool act = r < rows;
    const int rr = act ? r : 0;
    const A* vrow = parts + (size_t)np * 2 + rr;   // [np][rows] after the (m, s) pairs
    const double un0 = U_nom[rr];
    const A inf = A(INFINITY), il = A(1) / A(lambda);
    A m = inf, sw = A(0), acc = A(0);
    // fold (mp, sp, vp) into (m, sw, acc): a lower finite minimum rescales
    // what is held (by 0 while m is still +inf); an empty entry adds 0
    auto fold = [&](A mp, A sp, A vp) {
        const bool ok = mp < inf, lower = ok && mp < m;
        const A fr = lower ? merge_exp((mp - m) * il) : A(1);
        sw *= fr;
        acc *= fr;
        m = lower ? mp : m;
        const A f = ok ? merge_exp((m - mp) * il) : A(0);
        sw += f * sp;
        acc += f * vp;
    };
    // (m, s, V) of NB entries: their minimum, then the sums rescaled to it
    auto reduce = [&](const A* mv, const A* sv, const A* vv, int NB_, A& mb, A& sb, A& vb) {
        mb = inf;
        for (int u = 0; u < NB_; ++u) mb = mv[u] < mb ? mv[u] : mb;
        sb = A(0);
        vb = A(0);
        for (int u = 0; u < NB_; ++u) {
            const A f = mv[u] < inf ? merge_exp((mb - mv[u]) * il) : A(0);
            sb += f * sv[u];
            vb += f * vv[u];
        }
    };
    // the first batch runs on every thread (a slice past np holds only
    // empty entries), so the kernel arguments are all read up front
    constexpr int NB = 16;
    int p0 = sl;
    do {
        A mv[NB], sv[NB], vv[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int p = p0 + u * kMergeSlices, pc = p < np ? p : 0;
            mv[u] = parts[2 * pc];
            sv[u] = parts[2 * pc + 1];
            vv[u] = vrow[pc * rows];
        }
        // keep the batch's loads ahead of their first use (the scheduler
        // otherwise spreads them over the reduction, one wait each); slots
        // past np are marked empty only after it
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < NB; ++u) mv[u] = p0 + u * kMergeSlices < np ? mv[u] : inf;
        A mb, sb, vb;
        reduce(mv, sv, vv, NB, mb, sb, vb);
        fold(mb, sb, vb);
        p0 += NB * kMergeSlices;
    } while (p0 < np);
    shm[tid] = m;
    shs[tid] = sw;
    shv[tid] = acc;
    __syncthreads();
    if (sl != 0 || !act) return;
    {
        A mq[kMergeSlices], sq[kMergeSlices], vq[kMergeSlices];
#pragma unroll
        for (int q = 0; q < kMergeSlices; ++q) {
            mq[q] = shm[q * kMergeRows + rl];
            sq[q] = shs[q * kMergeRows + rl];
            vq[q] = shv[q * kMergeRows + rl];
        }
        reduce(mq, sq, vq, kMergeSlices, m, sw, acc);
    }
    const int t = r / NJ, jj = r % NJ;
    const double un = m < inf ? un0 + double(acc / sw) : un0;
    U_new[r] = un;
    if (U_shift) {
        if (t >= 1) U_shift[(t - 1) * NJ + jj] = un;
        if (t == T - 1) U_shift[t * NJ + jj] = un;
    }
    if (status && r == 0) *status = m < inf ? MPPI_OK : MPPI_ENONFINITE;
}

// Batched update (a13): many independent problems (own arm, cost, K, T,
// seed) in one persistent launch.  Work items are 64-sample tiles, ordered
// longest horizon first on the host; every wave pops items from a
// device-scope queue, rolls out its tile, writes the tile's Eq. 4 partial
// (noise regenerated from the Philox counters) and bumps its problem's
// counter; the wave that completes a problem merges that problem's
// partials.  The last wave to leave resets the queue, and every problem
// counter is reset by its merging wave, so the launch can be replayed (a
// captured graph) without clearing memory in between.
struct BatchProblem {
    const ModelM<float>* model;
    const CostM<float>* cost;
    const ModelM<double>* model64;   // the FP64 plant
    const CostM<double>* cost64;
    int K, T, force, acc64, coll;
    double lambda;
    int ntiles;
    int pad;
    long long u_off;      // into the packed [sum T][7] arrays
    long long k_off;      // into the packed costs
    long long part_off;   // into the partials buffer, in doubles
};

// COLL: some problem of the batch has the collision term (the collision
// rollout variants are compiled in only then).  Without it the kernel is
// built for two resident waves per SIMD (at most 256 registers per lane,
// some spilled to scratch): the second wave fills the dependency stalls of
// the first, 17 % faster on the 64-problem tick than one wave holding the
// whole register file.  The collision variants spill too much at that size
// and keep one wave per SIMD.
template <int W, bool COLL>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(COLL ? 1 : 2))) void batch_kernel(
    const BatchProblem* __restrict__ probs, const ModelM<float>* __restrict__ models,
    const int2* __restrict__ items, int nitems, unsigned int* queue, unsigned int* done, unsigned int* counters, const double* __restrict__ q,
    const double* __restrict__ qd, const double* __restrict__ target, const double* U_nom, double* U_new,
    double* U_shift, float* __restrict__ costs, int* __restrict__ status, const uint64_t* __restrict__ seeds,
    const uint64_t* __restrict__ tickp, int iter, int niter, double* __restrict__ parts)
{
    __shared__ CostM<float> Csh[W];
    __shared__ float Us[W][kMaxTBatch * NJ];
    __shared__ float tr[W][64 * kLdsRowPad];
    __shared__ double wl[W][64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t tick = (uint32_t)(*tickp * (uint64_t)niter + (uint64_t)iter);
    // Queue pops, completion counts and the exit count are atomics that every
    // lane executes (adding 1 on lane 0 and 0 elsewhere) with the result
    // taken from lane 0, so the control flow around them stays uniform: a
    // lane-0-only atomic inside this loop let the compiler split the loop
    // so that lanes 1..63 re-ran a tile with a stale item.
    for (;;) {
        const int item = __builtin_amdgcn_readfirstlane((int)atomicAdd(queue, lane == 0 ? 1u : 0u));
        if (item >= nitems) break;
        const int2 it = items[item];
        const BatchProblem& Pb = probs[it.x];
        const int T = Pb.T, K = Pb.K;
        wave_sync();
        wave_copy(&Csh[wid], Pb.cost, lane);
        for (int i = lane; i < T * NJ; i += 64) Us[wid][i] = float(U_nom[Pb.u_off + i]);
        wave_sync();
        // problem p's model is models[p] (== *Pb.model); read through the
        // restrict-qualified kernel argument at a uniform index it becomes
        // scalar loads, as in update_kernel (a pointer loaded from the
        // problem table is read with vector loads)
        const ModelM<float>& M = models[it.x];
        const CostM<float>& C = Csh[wid];
        const int k = it.y * 64 + lane;
        const uint64_t seed = seeds[it.x];
        float s = INFINITY;
        {
            TargetM<float> tg;
            make_target(target + (size_t)it.x * 13, tg);
            float q0[NJ], qd0[NJ], te[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                q0[j] = float(q[it.x * NJ + j]);
                qd0[j] = float(qd[it.x * NJ + j]);
                te[j] = 0.0f;
            }
            if (C.ext_mode == EXTW_CONST) const_ext_torque(M, C, q0, te);
            if (k < K) {
                float v;
                if (COLL && Pb.coll)
                    v = Pb.force ? rollout_sample<float, true, false, true>(M, C, tg, q0, qd0, te, Us[wid], T, seed,
                                                                            tick, (uint32_t)k, (float*)nullptr, 0)
                                 : rollout_sample<float, false, false, true>(M, C, tg, q0, qd0, te, Us[wid], T, seed,
                                                                             tick, (uint32_t)k, (float*)nullptr, 0);
                else
                    v = Pb.force ? rollout_sample<float, true>(M, C, tg, q0, qd0, te, Us[wid], T, seed, tick,
                                                               (uint32_t)k, (float*)nullptr, 0)
                                 : rollout_sample<float, false>(M, C, tg, q0, qd0, te, Us[wid], T, seed, tick,
                                                                (uint32_t)k, (float*)nullptr, 0);
                s = finite_(v) ? v : INFINITY;
                if (costs) costs[Pb.k_off + k] = s;
            }
        }
        const int P = 2 + T * NJ;
        double* pbase = parts + Pb.part_off;
        wave_sync();
        if (Pb.acc64)
            wave_partial<float, double>(s, lane, T, Pb.lambda, nullptr, C, seed, tick, (uint32_t)k, tr[wid],
                                        wl[wid], pbase + (size_t)it.y * P);
        else
            wave_partial<float, float>(s, lane, T, Pb.lambda, nullptr, C, seed, tick, (uint32_t)k, tr[wid],
                                       reinterpret_cast<float*>(wl[wid]),
                                       reinterpret_cast<float*>(pbase) + (size_t)it.y * P);
        __threadfence();
        const unsigned done_tiles =
            (unsigned)__builtin_amdgcn_readfirstlane((int)atomicAdd(&counters[it.x], lane == 0 ? 1u : 0u));
        if (done_tiles == (unsigned)(Pb.ntiles - 1)) {
            __threadfence();
            const double* un = U_nom + Pb.u_off;
            double* uw = U_new + Pb.u_off;
            double* us = U_shift ? U_shift + Pb.u_off : nullptr;
            int* st = status ? status + it.x : nullptr;
            if (Pb.acc64) wave_merge<double>(pbase, Pb.ntiles, T, Pb.lambda, un, uw, us, st, lane, wl[wid]);
            else
                wave_merge<float>(reinterpret_cast<const float*>(pbase), Pb.ntiles, T, Pb.lambda, un, uw, us, st,
                                  lane, reinterpret_cast<float*>(wl[wid]));
            if (lane == 0) counters[it.x] = 0u;
        }
    }
    // the last wave out resets the queue for the next launch
    __threadfence();
    const unsigned out = (unsigned)__builtin_amdgcn_readfirstlane((int)atomicAdd(done, lane == 0 ? 1u : 0u));
    if (out == gridDim.x * W - 1 && lane == 0) {
        *queue = 0u;
        *done = 0u;
        __threadfence();
    }
}

// Batched update with eight lanes per sample (mppi_batch_set_launch(b, 8,
// groups)): a workgroup of eight waves takes one 64-sample tile of the work
// list at a time, wave w the samples 8 w .. 8 w + 7 of the tile, each on a
// group of eight lanes running group_rollout (group.hpp; the dynamics and
// the cost of a step on one wave, the single-problem eight-lane update's
// arithmetic without its two-wave split).  The tile's Eq. 4 partial (noise
// regenerated per lane from the Philox counters, reduced over the eight
// samples of a wave by shuffles and over the waves through LDS), the
// problem counters, the merge by the workgroup that completes a problem and
// the queue reset by the last workgroup out follow batch_kernel at
// workgroup granularity: both kernels write the same partials and share
// the queue and counters (they never run concurrently on one batch).
constexpr int kBatchGroupWaves = 8;

template <typename A>
__device__ void group_tile_partial(const float* sS, A* wsm, A (*vs)[kGroupSteps * 8], int tid, int lane, int wave,
                                   int j, int grp, int T, double lambda, const CostM<float>& C,
                                   const GroupLink<float>& L, uint64_t seed, uint32_t tick, uint32_t k, A* part)
{
    const A inf = A(INFINITY), il = A(1) / A(lambda);
    A m = inf;
    for (int i = 0; i < 64; ++i) m = fmin(m, sS[i] < INFINITY ? A(sS[i]) : inf);
    if (tid < 64) wsm[tid] = sS[tid] < INFINITY ? exp((m - A(sS[tid])) * il) : A(0);
    __syncthreads();
    const A wgt = wsm[grp];
    float dr = 0.0f;
    for (int t0 = 0; t0 < T; t0 += kGroupSteps) {
        const int nt = min(kGroupSteps, T - t0);
        for (int tt = 0; tt < nt; ++tt) {
            const int t = t0 + tt;
            dr = group_noise_step(C, L, group_normal<float>(seed, tick, k, (uint32_t)t, j), dr, t);
            // over the wave's 8 samples (lane bits 0, 4, 5)
            A x = wgt * A(dr);
            x += __shfl_xor(x, 1);
            x += __shfl_xor(x, 16);
            x += __shfl_xor(x, 32);
            if ((lane & 0x31) == 0) vs[wave][tt * 8 + j] = x;
        }
        __syncthreads();
        for (int r = tid; r < nt * NJ; r += 64 * kBatchGroupWaves) {
            const int tt = r / NJ, jj = r % NJ;
            A acc = A(0);
#pragma unroll
            for (int w = 0; w < kBatchGroupWaves; ++w) acc += vs[w][tt * 8 + jj];
            part[2 + (t0 + tt) * NJ + jj] = acc;
        }
        __syncthreads();
    }
    if (tid == 0) {
        A st = A(0);
        for (int i = 0; i < 64; ++i) st += wsm[i];
        part[0] = m;
        part[1] = st;
    }
}

template <bool COLL>
__global__ __launch_bounds__(64 * kBatchGroupWaves) void batch_group_kernel(
    const BatchProblem* __restrict__ probs, const ModelM<float>* __restrict__ models,
    const int2* __restrict__ items, int nitems, unsigned int* queue, unsigned int* done, unsigned int* counters,
    const double* __restrict__ q, const double* __restrict__ qd, const double* __restrict__ target,
    const double* U_nom, double* U_new, double* U_shift, float* __restrict__ costs, int* __restrict__ status,
    const uint64_t* __restrict__ seeds, const uint64_t* __restrict__ tickp, int iter, int niter,
    double* __restrict__ parts)
{
    __shared__ float gx[kBatchGroupWaves * 8][kGxCount];
    __shared__ float Us[kMaxTBatch * NJ];
    __shared__ CostM<float> Csh;
    __shared__ float sS[64];
    __shared__ double wsm[64];
    __shared__ double vs[kBatchGroupWaves][kGroupSteps * 8];
    __shared__ int sItem, sDone;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = group_joint(lane), grp = wave * 8 + group_sample(lane);   // sample grp of the tile
    const uint32_t tick = (uint32_t)(*tickp * (uint64_t)niter + (uint64_t)iter);
    for (;;) {
        if (tid == 0) sItem = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int item = sItem;
        if (item >= nitems) break;
        const int2 it = items[item];
        const BatchProblem& Pb = probs[it.x];
        const int T = Pb.T, K = Pb.K;
        if (wave == 0) wave_copy(&Csh, Pb.cost, lane);
        for (int i = tid; i < T * NJ; i += 64 * kBatchGroupWaves) Us[i] = float(U_nom[Pb.u_off + i]);
        __syncthreads();
        // problem p's model through the restrict-qualified argument at a
        // uniform index (scalar loads), as in batch_kernel
        const ModelM<float>& M = models[it.x];
        const CostM<float>& C = Csh;
        const int k = it.y * 64 + grp;
        const uint64_t seed = seeds[it.x];
        GroupLink<float> L;
        group_link(M, C, j, L);
        const float grav[3] = {M.g[0], M.g[1], M.g[2]};
        TargetM<float> tg;
        make_target(target + (size_t)it.x * 13, tg);
        float q0 = 0.0f, qd0 = 0.0f, te = 0.0f;
        {
            float qa[NJ], qda[NJ], tea[NJ];
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                qa[i] = float(q[it.x * NJ + i]);
                qda[i] = float(qd[it.x * NJ + i]);
                tea[i] = 0.0f;
            }
            if (C.ext_mode == EXTW_CONST) const_ext_torque(M, C, qa, tea);
#pragma unroll
            for (int i = 0; i < NJ; ++i)
                if (i == j) { q0 = qa[i]; qd0 = qda[i]; te = tea[i]; }
        }
        // every group rolls out (samples past K too, storing nothing), so
        // the DPP moves always see a converged wave
        const DevGroup g{j, gx[grp]};
        float S;
        if (COLL && Pb.coll)
            S = Pb.force ? group_rollout<float, true, DevGroup, float, true>(g, L, C, tg, grav, q0, qd0, te, Us, T,
                                                                              seed, tick, (uint32_t)k, nullptr, 0, nullptr, 0, true)
                         : group_rollout<float, false, DevGroup, float, true>(g, L, C, tg, grav, q0, qd0, te, Us, T,
                                                                               seed, tick, (uint32_t)k, nullptr, 0, nullptr, 0, true);
        else
            S = Pb.force ? group_rollout<float, true, DevGroup, float>(g, L, C, tg, grav, q0, qd0, te, Us, T, seed,
                                                                       tick, (uint32_t)k, nullptr, 0, nullptr, 0, true)
                         : group_rollout<float, false, DevGroup, float>(g, L, C, tg, grav, q0, qd0, te, Us, T, seed,
                                                                        tick, (uint32_t)k, nullptr, 0, nullptr, 0, true);
        float sv = INFINITY;
        if (k < K) {
            sv = finite_(S) ? S : INFINITY;
            if (j == 0 && costs) costs[Pb.k_off + k] = sv;
        }
        if (j == 0) sS[grp] = sv;
        __syncthreads();
        double* pbase = parts + Pb.part_off;
        const int P = 2 + T * NJ;
        if (Pb.acc64)
            group_tile_partial<double>(sS, wsm, vs, tid, lane, wave, j, grp, T, Pb.lambda, C, L, seed, tick,
                                       (uint32_t)k, pbase + (size_t)it.y * P);
        else
            group_tile_partial<float>(sS, reinterpret_cast<float*>(wsm),
                                      reinterpret_cast<float (*)[kGroupSteps * 8]>(vs), tid, lane, wave, j, grp, T,
                                      Pb.lambda, C, L, seed, tick, (uint32_t)k,
                                      reinterpret_cast<float*>(pbase) + (size_t)it.y * P);
        __threadfence();
        __syncthreads();
        if (tid == 0) sDone = (int)atomicAdd(&counters[it.x], 1u);
        __syncthreads();
        if (sDone == Pb.ntiles - 1) {
            __threadfence();
            if (wave == 0) {
                const double* un = U_nom + Pb.u_off;
                double* uw = U_new + Pb.u_off;
                double* us = U_shift ? U_shift + Pb.u_off : nullptr;
                int* st = status ? status + it.x : nullptr;
                if (Pb.acc64) wave_merge<double>(pbase, Pb.ntiles, T, Pb.lambda, un, uw, us, st, lane, wsm);
                else
                    wave_merge<float>(reinterpret_cast<const float*>(pbase), Pb.ntiles, T, Pb.lambda, un, uw, us,
                                      st, lane, reinterpret_cast<float*>(wsm));
                if (lane == 0) counters[it.x] = 0u;
            }
        }
        __syncthreads();
    }
    // the last workgroup out resets the queue for the next launch
    if (tid == 0) {
        __threadfence();
        const unsigned out = atomicAdd(done, 1u);
        if (out == gridDim.x - 1) {
            *queue = 0u;
            *done = 0u;
            __threadfence();
        }
    }
}

__global__ void advance_tick_kernel(uint64_t* tick)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *tick += 1;
}

__global__ void set_tick_kernel(uint64_t* tick, uint64_t v)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *tick = v;
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

// zero-order hold of u (clamped to the torque limits) over dt in
// `substeps` semi-implicit Euler steps of the FP64 dynamics, with the cost's
// external-wrench model and, when `wrench` is non-null, a further world
// wrench [force; moment] at the EE point (a disturbance the controller does
// not model), J(q)^T wrench at the state of every substep
__device__ void plant_advance(const ModelM<double>& M, const CostM<double>& C, double* q, double* qd,
                              const double* u, double dt, int substeps, const double* wrench)
{
    double tau[NJ], qq[NJ], qv[NJ], W[6];
    for (int j = 0; j < NJ; ++j) {
        double lim = M.L[j].taumax;
        tau[j] = fmin(fmax(u[j], -lim), lim);
        qq[j] = q[j];
        qv[j] = qd[j];
    }
    for (int c = 0; c < 6; ++c) W[c] = wrench ? wrench[c] : 0.0;
    const int ext = C.ext_mode == EXTW_WALL ? EXTW_WALL : (C.ext_mode == EXTW_CONST ? EXTW_CONST : EXTW_NONE);
    const double h = dt / substeps;
    for (int s = 0; s < substeps; ++s) {
        double ts[NJ];
        if (wrench) {
            ee_wrench_torque(M, qq, W, ts);
            for (int j = 0; j < NJ; ++j) ts[j] += tau[j];
        } else {
            for (int j = 0; j < NJ; ++j) ts[j] = tau[j];
        }
        StepOut<double> o;
        dyn_step<double, false>(M, C, ext, qq, qv, ts, ts, o);
        for (int j = 0; j < NJ; ++j) {
            qv[j] += o.qdd[j] * h;
            qq[j] += qv[j] * h;
        }
    }
    for (int j = 0; j < NJ; ++j) { q[j] = qq[j]; qd[j] = qv[j]; }
}

__global__ void plant_kernel(const ModelM<double>* __restrict__ Mp, const CostM<double>* __restrict__ Cp,
                             double* q, double* qd, const double* __restrict__ u, double dt, int substeps,
                             const double* __restrict__ wrench)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    plant_advance(*Mp, *Cp, q, qd, u, dt, substeps, wrench);
}

// EE pose of n states (FP64): position and the unit quaternion (w, x, y, z)
// of the EE frame, w >= 0; one thread per state.  The quaternion is taken
// from the rotation matrix by its largest diagonal combination (Shepperd's
// method), which keeps the square root away from zero.
__global__ void ee_pose_kernel(const ModelM<double>* __restrict__ Mp, const double* __restrict__ q, int n,
                               double* __restrict__ pose)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const ModelM<double>& M = *Mp;
    double qi[NJ], p[3], Rn[9];
    for (int j = 0; j < NJ; ++j) qi[j] = q[i * NJ + j];
    fk_ee(M, qi, p, Rn, (double*)nullptr, (double*)nullptr);
    double Re[9];
    mm3(Rn, M.Ree, Re);
    const double tr = Re[0] + Re[4] + Re[8];
    double w, x, y, z;
    if (tr >= Re[0] && tr >= Re[4] && tr >= Re[8]) {
        const double r = sqrt(1.0 + tr), s = 0.5 / r;
        w = 0.5 * r; x = (Re[7] - Re[5]) * s; y = (Re[2] - Re[6]) * s; z = (Re[3] - Re[1]) * s;
    } else if (Re[0] >= Re[4] && Re[0] >= Re[8]) {
        const double r = sqrt(1.0 + Re[0] - Re[4] - Re[8]), s = 0.5 / r;
        x = 0.5 * r; w = (Re[7] - Re[5]) * s; y = (Re[1] + Re[3]) * s; z = (Re[2] + Re[6]) * s;
    } else if (Re[4] >= Re[8]) {
        const double r = sqrt(1.0 - Re[0] + Re[4] - Re[8]), s = 0.5 / r;
        y = 0.5 * r; w = (Re[2] - Re[6]) * s; x = (Re[1] + Re[3]) * s; z = (Re[5] + Re[7]) * s;
    } else {
        const double r = sqrt(1.0 - Re[0] - Re[4] + Re[8]), s = 0.5 / r;
        z = 0.5 * r; w = (Re[3] - Re[1]) * s; x = (Re[2] + Re[6]) * s; y = (Re[5] + Re[7]) * s;
    }
    const double sg = w < 0.0 ? -1.0 : 1.0;
    double* o = pose + (size_t)i * 7;
    o[0] = p[0]; o[1] = p[1]; o[2] = p[2];
    o[3] = sg * w; o[4] = sg * x; o[5] = sg * y; o[6] = sg * z;
}

// one workgroup per problem of a batch: the first row of its U_new
__global__ void batch_plant_kernel(const BatchProblem* __restrict__ probs, int n, double* q, double* qd,
                                   const double* __restrict__ U_new, double dt, int substeps)
{
    const int p = blockIdx.x;
    if (p >= n || threadIdx.x != 0) return;
    const BatchProblem& Pb = probs[p];
    plant_advance(*Pb.model64, *Pb.cost64, q + p * NJ, qd + p * NJ, U_new + Pb.u_off, dt, substeps, nullptr);
}

// Warm start after s horizon steps of elapsed time (solver period != dt):
// the sequence read as piecewise constant in time (row i held over
// [i, i+1) steps, the last row held past the horizon), averaged over
// [t + s, t + s + 1):  out[t] = (1 - f) U[min(t+m, T-1)] + f U[min(t+m+1, T-1)]
// with m = floor(s), f = s - m (f = 0 copies the row, so s = 1 is the
// one-step shift bit for bit).
__device__ void warm_start_rows(const double* U, double* out, int T, double s, int tid, int nthreads)
{
    const double mf = floor(s), f = s - mf;
    const int m = (int)mf;
    for (int r = tid; r < T * NJ; r += nthreads) {
        const int t = r / NJ, j = r - t * NJ;
        const int i0 = min(t + m, T - 1), i1 = min(t + m + 1, T - 1);
        const double a = U[i0 * NJ + j];
        out[r] = f == 0.0 ? a : (1.0 - f) * a + f * U[i1 * NJ + j];
    }
}

__global__ void warm_start_kernel(const double* __restrict__ U, double* __restrict__ out, int T, double s)
{
    warm_start_rows(U, out, T, s, threadIdx.x, blockDim.x);
}

// one workgroup per problem of a batch (packed layout)
__global__ void batch_warm_start_kernel(const BatchProblem* __restrict__ probs, int n, const double* __restrict__ U,
                                        double* __restrict__ out, double s)
{
    const int p = blockIdx.x;
    if (p >= n) return;
    const BatchProblem& Pb = probs[p];
    warm_start_rows(U + Pb.u_off, out + Pb.u_off, Pb.T, s, threadIdx.x, blockDim.x);
}

// Noise-free costs of two sequences from one state (lane 0: the current
// nominal, lane 1: the candidate; the sampling scales are zeroed in the LDS
// copy of the cost, so v_t = u_t exactly); the candidate replaces the
// nominal only when it costs less.
template <typename R, bool FORCE, bool COLL>
__device__ void select_two(const ModelM<R>& Mg, const CostM<R>& Cg, const double* q0, const double* qd0,
                           const double* target, double* U_nom, const double* U_cand, int T, double* costs,
                           ModelM<R>& Msh, CostM<R>& Csh, R* Us, R* sc)
{
    const int lane = threadIdx.x & 63;
    wave_copy(&Msh, &Mg, lane);
    wave_copy(&Csh, &Cg, lane);
    for (int i = lane; i < T * NJ; i += 64) {
        Us[i] = R(U_nom[i]);
        Us[kMaxT * NJ + i] = R(U_cand[i]);
    }
    wave_sync();
    if (lane < NJ) Csh.sigma[lane] = Csh.sig_c[lane] = R(0);
    wave_sync();
    if (lane < 2) {
        TargetM<R> tg;
        make_target(target, tg);
        R q[NJ], qd[NJ], te[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) { q[j] = R(q0[j]); qd[j] = R(qd0[j]); te[j] = R(0); }
        if (Csh.ext_mode == EXTW_CONST) const_ext_torque(Msh, Csh, q, te);
        const R v = rollout_sample<R, FORCE, false, COLL>(Msh, Csh, tg, q, qd, te, Us + lane * kMaxT * NJ, T, 0ull, 0u, 0u,
                                             (R*)nullptr, 0);
        sc[lane] = finite_(v) ? v : R(INFINITY);
    }
    wave_sync();
    const bool take = sc[1] < sc[0];
    if (take)
        for (int i = lane; i < T * NJ; i += 64) U_nom[i] = U_cand[i];
    if (costs && lane < 2) costs[lane] = double(sc[lane]);
}

template <typename R, bool FORCE, bool COLL>
__global__ __launch_bounds__(64) void select_kernel(const ModelM<R>* __restrict__ Mp, const CostM<R>* __restrict__ Cp,
                                                    const double* q0, const double* qd0, const double* target,
                                                    double* U_nom, const double* U_cand, int T, double* costs)
{
    __shared__ ModelM<R> Msh;
    __shared__ CostM<R> Csh;
    __shared__ R Us[2 * kMaxT * NJ];
    __shared__ R sc[2];
    select_two<R, FORCE, COLL>(*Mp, *Cp, q0, qd0, target, U_nom, U_cand, T, costs, Msh, Csh, Us, sc);
}

__global__ __launch_bounds__(64) void batch_select_kernel(const BatchProblem* __restrict__ probs, int n,
                                                          const double* q, const double* qd, const double* target,
                                                          double* U_nom, const double* U_cand, double* costs)
{
    __shared__ ModelM<float> Msh;
    __shared__ CostM<float> Csh;
    __shared__ float Us[2 * kMaxT * NJ];
    __shared__ float sc[2];
    const int p = blockIdx.x;
    if (p >= n) return;
    const BatchProblem& Pb = probs[p];
    double* c = costs ? costs + 2 * p : nullptr;
    const double* qp = q + p * NJ;
    const double* qdp = qd + p * NJ;
    const double* tp = target + (size_t)p * 13;
    double* un = U_nom + Pb.u_off;
    const double* uc = U_cand + Pb.u_off;
    if (Pb.coll) {
        if (Pb.force) select_two<float, true, true>(*Pb.model, *Pb.cost, qp, qdp, tp, un, uc, Pb.T, c, Msh, Csh, Us, sc);
        else select_two<float, false, true>(*Pb.model, *Pb.cost, qp, qdp, tp, un, uc, Pb.T, c, Msh, Csh, Us, sc);
    } else {
        if (Pb.force) select_two<float, true, false>(*Pb.model, *Pb.cost, qp, qdp, tp, un, uc, Pb.T, c, Msh, Csh, Us, sc);
        else select_two<float, false, false>(*Pb.model, *Pb.cost, qp, qdp, tp, un, uc, Pb.T, c, Msh, Csh, Us, sc);
    }
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

template <typename R, typename A, bool FORCE, bool EXPLICIT, bool COLL>
static hipError_t update_t(const UpdateArgs& a, hipStream_t s)
{
    dim3 grid((a.K + kRolloutBlock - 1) / kRolloutBlock);
    const size_t rows = (size_t)a.T * NJ;
    const size_t tile = rows * kLdsRowPad * sizeof(R);
    const int lds_noise = a.merge && tile <= (size_t)kMaxDynLds;
    const size_t dyn = lds_noise ? tile : (a.merge ? 64 * kLdsRowPad * sizeof(R) : 0);
    // global noise: always for rollouts-only launches, otherwise only when
    // the caller asked for it
    R* noise = (R*)a.noise;
    if (a.merge && !a.want_noise) noise = nullptr;
    hipLaunchKernelGGL((update_kernel<R, A, FORCE, EXPLICIT, COLL>), grid, dim3(kRolloutBlock), dyn, s,
                       (const ModelM<R>*)a.model, (const CostM<R>*)a.cost, a.q0, a.qd0, a.target, a.U_nom,
                       a.seed, (uint32_t)a.tick, a.K, a.T, a.lambda, noise, (R*)a.costs, a.merge, lds_noise,
                       (A*)a.parts, a.counter, a.U_new, a.U_shift, a.status);
    return hipGetLastError();
}

template <typename A, bool FORCE, bool COLL> static hipError_t update_split_t(const UpdateArgs& a, hipStream_t s)
{
    dim3 grid((a.K + 63) / 64);
    const size_t rows = (size_t)a.T * NJ;
    const size_t tile = rows * kLdsRowPad * sizeof(float);
    const int lds_noise = a.merge && tile <= (size_t)kMaxDynLds;
    const size_t dyn = lds_noise ? tile : (a.merge ? 64 * kLdsRowPad * sizeof(float) : 0);
    float* noise = (float*)a.noise;
    if (a.merge && !a.want_noise) noise = nullptr;
    hipLaunchKernelGGL((update_split_kernel<A, FORCE, COLL>), grid, dim3(128), dyn, s, (const ModelM<float>*)a.model,
                       (const CostM<float>*)a.cost, a.q0, a.qd0, a.target, a.U_nom, a.seed, (uint32_t)a.tick, a.K,
                       a.T, a.lambda, noise, (float*)a.costs, a.merge, lds_noise, (A*)a.parts, a.counter, a.U_new,
                       a.U_shift, a.status);
    return hipGetLastError();
}

template <typename A, bool FORCE, bool COLL> static hipError_t update_group_t(const UpdateArgs& a, hipStream_t s)
{
    dim3 grid((a.K + kGroupSamples - 1) / kGroupSamples);
    float* noise = (float*)a.noise;
    if (a.merge && !a.want_noise) noise = nullptr;
    const size_t tile = (size_t)a.T * NJ * kGroupTile * sizeof(float);
    const int lds_noise = a.merge && tile <= (size_t)kMaxDynLds;
    hipLaunchKernelGGL((update_group_kernel<A, FORCE, COLL>), grid, dim3(kGroupThreads), lds_noise ? tile : 0, s,
                       (const ModelM<float>*)a.model, (const CostM<float>*)a.cost, a.q0, a.qd0, a.target, a.U_nom,
                       a.seed, (uint32_t)a.tick, a.K, a.T, a.lambda, noise, (float*)a.costs, a.merge, lds_noise,
                       (A*)a.parts);
    if (a.merge)
        hipLaunchKernelGGL((group_merge_kernel<A>), dim3((a.T * NJ + kMergeRows - 1) / kMergeRows),
                           dim3(kGroupThreads), 0, s, (const A*)a.parts,
                           (int)grid.x, a.T, a.lambda, a.U_nom, a.U_new, a.U_shift, a.status);
    return hipGetLastError();
}

template <bool EXPLICIT, bool COLL>
static hipError_t update_dispatch(int precision, bool acc64, bool force, const UpdateArgs& a, hipStream_t s)
{
    if (!EXPLICIT && a.waves_per_group == 8 && precision == MPPI_FP32) {
        if (force) return acc64 ? update_group_t<double, true, COLL>(a, s) : update_group_t<float, true, COLL>(a, s);
        return acc64 ? update_group_t<double, false, COLL>(a, s) : update_group_t<float, false, COLL>(a, s);
    }
    if (a.waves_per_group == 8) {   // the two-wave launch where groups do not apply
        UpdateArgs b = a;
        b.waves_per_group = 2;
        return update_dispatch<EXPLICIT, COLL>(precision, acc64, force, b, s);
    }
    if (!EXPLICIT && a.waves_per_group == 2 && precision == MPPI_FP32) {
        if (force) return acc64 ? update_split_t<double, true, COLL>(a, s) : update_split_t<float, true, COLL>(a, s);
        return acc64 ? update_split_t<double, false, COLL>(a, s) : update_split_t<float, false, COLL>(a, s);
    }
    if (precision == MPPI_FP64)
        return force ? update_t<double, double, true, EXPLICIT, COLL>(a, s)
                     : update_t<double, double, false, EXPLICIT, COLL>(a, s);
    if (acc64)
        return force ? update_t<float, double, true, EXPLICIT, COLL>(a, s)
                     : update_t<float, double, false, EXPLICIT, COLL>(a, s);
    return force ? update_t<float, float, true, EXPLICIT, COLL>(a, s) : update_t<float, float, false, EXPLICIT, COLL>(a, s);
}

hipError_t launch_update(int precision, bool acc64, bool force, const UpdateArgs& a, hipStream_t s)
{
    if (a.T < 1 || a.T > kMaxT || a.K < 1) return hipErrorInvalidValue;
    const bool ex = a.dynamics == MPPI_DYN_EXPLICIT_M;
    if (a.collision)
        return ex ? update_dispatch<true, true>(precision, acc64, force, a, s)
                  : update_dispatch<false, true>(precision, acc64, force, a, s);
    return ex ? update_dispatch<true, false>(precision, acc64, force, a, s)
              : update_dispatch<false, false>(precision, acc64, force, a, s);
}

size_t update_parts_bytes(int K, int T)
{
    // one partial per workgroup: 64 samples, or kGroupSamples with lane groups
    return (size_t)((K + kGroupSamples - 1) / kGroupSamples) * (2 + (size_t)T * NJ) * sizeof(double);
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

template <int W, bool COLL> static hipError_t batch_t(const BatchArgs& a, int groups, hipStream_t s)
{
    hipLaunchKernelGGL((batch_kernel<W, COLL>), dim3(groups), dim3(64 * W), 0, s, (const BatchProblem*)a.probs,
                       (const ModelM<float>*)a.models, (const int2*)a.items, a.nitems, a.queue, a.done, a.counters,
                       a.q, a.qd, a.target, a.U_nom, a.U_new, a.U_shift, a.costs, a.status, a.seeds, a.tick,
                       a.iter, a.niter, a.parts);
    return hipGetLastError();
}

template <bool COLL> static hipError_t batch_group_t(const BatchArgs& a, int groups, hipStream_t s)
{
    hipLaunchKernelGGL((batch_group_kernel<COLL>), dim3(groups), dim3(64 * kBatchGroupWaves), 0, s,
                       (const BatchProblem*)a.probs, (const ModelM<float>*)a.models, (const int2*)a.items, a.nitems,
                       a.queue, a.done, a.counters, a.q, a.qd, a.target, a.U_nom, a.U_new, a.U_shift, a.costs,
                       a.status, a.seeds, a.tick, a.iter, a.niter, a.parts);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& a, int waves_per_group, int groups, hipStream_t s)
{
    if (groups < 1 || a.nitems < 1) return hipErrorInvalidValue;
    switch (waves_per_group) {
    case 8: return a.collision ? batch_group_t<true>(a, groups, s) : batch_group_t<false>(a, groups, s);
    case 1: return a.collision ? batch_t<1, true>(a, groups, s) : batch_t<1, false>(a, groups, s);
    case 2: return a.collision ? batch_t<2, true>(a, groups, s) : batch_t<2, false>(a, groups, s);
    case 4: return a.collision ? batch_t<4, true>(a, groups, s) : batch_t<4, false>(a, groups, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_advance_tick(uint64_t* tick, hipStream_t s)
{
    hipLaunchKernelGGL(advance_tick_kernel, dim3(1), dim3(64), 0, s, tick);
    return hipGetLastError();
}

hipError_t launch_set_tick(uint64_t* tick, uint64_t v, hipStream_t s)
{
    hipLaunchKernelGGL(set_tick_kernel, dim3(1), dim3(64), 0, s, tick, v);
    return hipGetLastError();
}

size_t batch_problem_bytes() { return sizeof(BatchProblem); }

void fill_batch_problem(void* dst, const void* model, const void* cost, const void* model64, const void* cost64,
                        int K, int T, int force, int acc64, int coll, double lambda, int ntiles, long long u_off,
                        long long k_off, long long part_off)
{
    BatchProblem p;
    p.model = (const ModelM<float>*)model;
    p.cost = (const CostM<float>*)cost;
    p.model64 = (const ModelM<double>*)model64;
    p.cost64 = (const CostM<double>*)cost64;
    p.K = K; p.T = T; p.force = force; p.acc64 = acc64; p.coll = coll;
    p.lambda = lambda; p.ntiles = ntiles; p.pad = 0;
    p.u_off = u_off; p.k_off = k_off; p.part_off = part_off;
    memcpy(dst, &p, sizeof p);
}

hipError_t launch_plant(const ModelM<double>* M, const CostM<double>* C, double* q, double* qd,
                        const double* u, double dt, int substeps, const double* wrench, hipStream_t s)
{
    hipLaunchKernelGGL(plant_kernel, dim3(1), dim3(64), 0, s, M, C, q, qd, u, dt, substeps, wrench);
    return hipGetLastError();
}

hipError_t launch_ee_pose(const ModelM<double>* M, const double* q, int n, double* pose, hipStream_t s)
{
    hipLaunchKernelGGL(ee_pose_kernel, dim3((n + 63) / 64), dim3(64), 0, s, M, q, n, pose);
    return hipGetLastError();
}

hipError_t launch_batch_plant(const void* probs, int n, double* q, double* qd, const double* U_new, double dt,
                              int substeps, hipStream_t s)
{
    hipLaunchKernelGGL(batch_plant_kernel, dim3(n), dim3(64), 0, s, (const BatchProblem*)probs, n, q, qd, U_new,
                       dt, substeps);
    return hipGetLastError();
}

hipError_t launch_warm_start(const double* U, double* out, int T, double shift, hipStream_t s)
{
    if (T < 1 || T > kMaxT) return hipErrorInvalidValue;
    hipLaunchKernelGGL(warm_start_kernel, dim3(1), dim3(256), 0, s, U, out, T, shift);
    return hipGetLastError();
}

hipError_t launch_batch_warm_start(const void* probs, int n, const double* U, double* out, double shift,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(batch_warm_start_kernel, dim3(n), dim3(64), 0, s, (const BatchProblem*)probs, n, U, out,
                       shift);
    return hipGetLastError();
}

hipError_t launch_select(int precision, bool force, bool coll, const void* model, const void* cost,
                         const double* q0, const double* qd0, const double* target, double* U_nom,
                         const double* U_cand, int T, double* costs, hipStream_t s)
{
    if (T < 1 || T > kMaxT) return hipErrorInvalidValue;
    if (precision == MPPI_FP64) {
        auto k = coll ? (force ? select_kernel<double, true, true> : select_kernel<double, false, true>)
                      : (force ? select_kernel<double, true, false> : select_kernel<double, false, false>);
        hipLaunchKernelGGL(k, dim3(1), dim3(64), 0, s, (const ModelM<double>*)model, (const CostM<double>*)cost, q0,
                           qd0, target, U_nom, U_cand, T, costs);
    } else {
        auto k = coll ? (force ? select_kernel<float, true, true> : select_kernel<float, false, true>)
                      : (force ? select_kernel<float, true, false> : select_kernel<float, false, false>);
        hipLaunchKernelGGL(k, dim3(1), dim3(64), 0, s, (const ModelM<float>*)model, (const CostM<float>*)cost, q0,
                           qd0, target, U_nom, U_cand, T, costs);
    }
    return hipGetLastError();
}

hipError_t launch_batch_select(const void* probs, int n, const double* q, const double* qd, const double* target,
                               double* U_nom, const double* U_cand, double* costs, hipStream_t s)
{
    hipLaunchKernelGGL(batch_select_kernel, dim3(n), dim3(64), 0, s, (const BatchProblem*)probs, n, q, qd, target,
                       U_nom, U_cand, costs);
    return hipGetLastError();
}

}  // namespace mppi
