// launch.hpp -- host-side launchers of the kernels in kernels.hip (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "dyn.hpp"
#include "mppi.h"

namespace mppi {

struct RolloutArgs {
    const void* model;      // ModelM<R>* (device)
    const void* cost;       // CostM<R>* (device)
    const double* q0;
    const double* qd0;
    const double* target;   // 13 doubles
    const double* U_nom;    // [T][7]
    uint64_t seed;
    uint64_t tick;
    int K, T;
    void* noise;            // R [T][7][K]
    void* costs;            // R [K]
};

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

hipError_t launch_prep_model(const mppi_robot_params* d_raw, ModelM<float>* d_mf, ModelM<double>* d_md,
                             hipStream_t s);
// precision: MPPI_FP32 / MPPI_FP64; force: the force-cost instantiation
hipError_t launch_rollout(int precision, bool force, const RolloutArgs& a, hipStream_t s);
// acc64: accumulate the weights and sums in FP64
hipError_t launch_weights(int precision, bool acc64, const WeightsArgs& a, hipStream_t s);
hipError_t launch_plant(const ModelM<double>* M, const CostM<double>* C, double* q, double* qd,
                        const double* u, double dt, int substeps, hipStream_t s);

constexpr int kRolloutBlock = 64;
constexpr int kWeightsBlock = 256;
constexpr int kWeightsRows = 2;
constexpr int kMaxT = 256;

}  // namespace mppi
