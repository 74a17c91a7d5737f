// launch.hpp -- host-side launchers of the kernels in kernels.hip (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "dyn.hpp"
#include "mppi.h"

namespace mppi {

struct WeightsArgs {
    const void* costs;      // R [K]
    const void* noise;      // R [T][7][K]
    const double* U_nom;
    double* U_new;
    double* U_shift;        // may be null
    int* status;            // may be null
    int K, T;
    double lambda;
};

struct UpdateArgs {
    const void* model;
    const void* cost;
    const double* q0;
    const double* qd0;
    const double* target;
    const double* U_nom;
    uint64_t seed;
    uint64_t tick;
    int K, T;
    double lambda;
    void* noise;            // R [T][7][K]
    void* costs;            // R [K]
    int merge;              // 0: rollouts only
    int want_noise;         // the caller asked for the noise (global copy)
    void* parts;            // A [ceil(K/64)][2 + 7T]
    unsigned int* counter;  // zero before the launch; the kernel leaves it zero
    double* U_new;
    double* U_shift;
    int* status;
    int dynamics;           // mppi_dynamics
    int collision;          // the collision term is on (n_pairs > 0)
    int waves_per_group;    // 2: the two-wave split update (FP32 articulated-body
                            // rollouts); 8: eight lanes per sample (FP32, no
                            // collision term; otherwise as 2); else 1
};

// One fused launch: rollouts, per-wave Eq. 4 partials, last-block merge.
hipError_t launch_update(int precision, bool acc64, bool force, const UpdateArgs& a, hipStream_t s);
size_t update_parts_bytes(int K, int T);

struct BatchArgs {
    const void* probs;      // BatchProblem [n] (device)
    const void* models;     // ModelM<float> [n] (device): problem p's model
    const void* items;      // int2 [nitems]: (problem, tile), in schedule order
    int nitems;
    unsigned int* queue;    // zero before the first launch; the kernel leaves it zero
    unsigned int* done;
    unsigned int* counters; // [n], zero; each reset by the problem's merging wave
    const double* q;        // [n][7]
    const double* qd;       // [n][7]
    const double* target;   // [n][13]
    const double* U_nom;    // packed [sum T][7]
    double* U_new;
    double* U_shift;        // may be null
    float* costs;           // packed [sum K], may be null
    int* status;            // [n], may be null
    const uint64_t* seeds;  // [n]
    const uint64_t* tick;   // [1] (device)
    double* parts;          // partials, sized by the host
    int collision;          // some problem has the collision term
    int iter, niter;        // iteration iter of niter: Philox tick word = *tick * niter + iter
};

// Persistent batched update: `groups` workgroups of `waves_per_group` waves.
hipError_t launch_batch(const BatchArgs& a, int waves_per_group, int groups, hipStream_t s);
hipError_t launch_advance_tick(uint64_t* tick, hipStream_t s);
hipError_t launch_set_tick(uint64_t* tick, uint64_t v, hipStream_t s);
size_t batch_problem_bytes();
void fill_batch_problem(void* dst, const void* model, const void* cost, const void* model64, const void* cost64,
                        int K, int T, int force, int acc64, int coll, double lambda, int ntiles, long long u_off,
                        long long k_off, long long part_off);
hipError_t launch_batch_plant(const void* probs, int n, double* q, double* qd, const double* U_new, double dt,
                              int substeps, hipStream_t s);
// warm start after `shift` horizon steps (0 <= shift), [T][7] or packed
hipError_t launch_warm_start(const double* U, double* out, int T, double shift, hipStream_t s);
hipError_t launch_batch_warm_start(const void* probs, int n, const double* U, double* out, double shift,
                                   hipStream_t s);
hipError_t launch_batch_select(const void* probs, int n, const double* q, const double* qd, const double* target,
                               double* U_nom, const double* U_cand, double* costs, hipStream_t s);
// model/cost: ModelM<R>/CostM<R> of the rollout precision
hipError_t launch_select(int precision, bool force, bool coll, const void* model, const void* cost,
                         const double* q0, const double* qd0, const double* target, double* U_nom,
                         const double* U_cand, int T, double* costs, hipStream_t s);

hipError_t launch_prep_model(const mppi_robot_params* d_raw, ModelM<float>* d_mf, ModelM<double>* d_md,
                             hipStream_t s);
// acc64: accumulate the weights and sums in FP64
hipError_t launch_weights(int precision, bool acc64, const WeightsArgs& a, hipStream_t s);
// wrench: device [6] world wrench at the EE point added to the plant's
// external model, or null
hipError_t launch_plant(const ModelM<double>* M, const CostM<double>* C, double* q, double* qd,
                        const double* u, double dt, int substeps, const double* wrench, hipStream_t s);
// EE position and quaternion (w >= 0) of n states: pose [n][7]
hipError_t launch_ee_pose(const ModelM<double>* M, const double* q, int n, double* pose, hipStream_t s);

constexpr int kRolloutBlock = 64;
constexpr int kWeightsBlock = 256;
constexpr int kWeightsRows = 2;
constexpr int kMaxT = 256;
constexpr int kMaxTBatch = 64;   // horizon limit of the batched kernel

}  // namespace mppi
