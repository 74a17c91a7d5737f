// mlp.hpp -- the proposal network's device layout and launchers (internal).
//
// Network: 21 -> 256 -> 256 -> 256 -> 126, tanh-GELU on the hidden layers,
// BF16 weights and activations, FP32 accumulation (MFMA), FP32 biases, FP32
// master weights for Adam.  Flat parameter order (the C ABI's): W_1 [256][21],
// b_1, W_2 [256][256], b_2, W_3 [256][256], b_3, W_4 [126][256], b_4.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mppi {

constexpr int kMlpIn = 21, kMlpInPad = 32, kMlpHid = 256, kMlpOut = 126, kMlpOutPad = 128;
constexpr int kMlpRows = 64;      // batch granularity: training buffers and batches padded to it
constexpr int kMlpWgRows = 16;    // states per forward workgroup (one matrix-core row tile)
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHid * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpHid * kMlpHid;
constexpr int kOffW4 = kOffB3 + kMlpHid;
constexpr int kOffB4 = kOffW4 + kMlpOut * kMlpHid;
constexpr int kMlpParams = kOffB4 + kMlpOut;
static_assert(kMlpParams == 169598, "parameter count");

// Device buffers of one network.  Weight copies are BF16 bit patterns:
// W1 [256][32] (columns 21..31 zero), W2, W3 [256][256], W4 [128][256]
// (rows 126, 127 zero); the transposes W2t, W3t [256][256] and W4t
// [256][128] (columns 126, 127 zero) feed the backward products.
// Training scratch holds one batch of up to Bp rows (a multiple of 64):
// activations a_l and backward signals e_l stored transposed ([features][Bp],
// BF16) for the weight-gradient contraction over the batch.  Every one of
// these [N][K] matrices is stored in matrix-core operand order (16 x 32
// fragments of 1 KB, mlp.hip frag_index), not row-major.  The
// pre-activations that GELU' needs stay in the registers of the thread that
// computed them.
struct MlpDev {
    float* theta;     // [P] FP32 master parameters
    float* m;         // [P] Adam first moment
    float* v;         // [P] Adam second moment
    float* grad;      // [P] last gradient
    uint16_t* W1;
    uint16_t* W2;
    uint16_t* W3;
    uint16_t* W4;
    uint16_t* W2t;
    uint16_t* W3t;
    uint16_t* W4t;
    uint16_t* aT0;    // [32][Bp]
    uint16_t* aT1;    // [256][Bp]
    uint16_t* aT2;
    uint16_t* aT3;
    uint16_t* eT1;    // [256][Bp]
    uint16_t* eT2;
    uint16_t* eT3;
    uint16_t* eT4;    // [128][Bp]
    float* lossp;     // [Bp / 16] per-workgroup sums of squared residuals
    const double* scale;   // [21]: q_max[7], qd_max[7], then 7 torque limits
    int Bp;
};

// Bytes of each buffer for a batch capacity Bp (host helper).
size_t mlp_scratch_bytes(int Bp);
// Lays the buffers out in one allocation of mlp_scratch_bytes(Bp) bytes.
void mlp_carve(MlpDev& d, void* base, int Bp);

// Forward for B rows (B <= d.Bp) of the features X [B][21], or (X null,
// inference only) of the features of the states q [B][7], qd [B][7],
// target [B][13], encoded in the same launch.  Inference: Ytgt == nullptr;
// writes Y [B][126] and/or U [B][u_stride] = tau_max * y (either may be
// null).  Training: Ytgt [B][126] given; also stores the activations, the
// pre-activations and the backward signals of the MSE loss, and the
// per-workgroup loss sums.
hipError_t launch_mlp_forward(const MlpDev& d, const float* X, int B, const float* Ytgt, float* Y, double* U,
                              int u_stride, hipStream_t s, const double* q = nullptr, const double* qd = nullptr,
                              const double* target = nullptr);
// One Adam step (update != 0) with c1 = 1 / (1 - beta1^t), c2 = 1 / (1 -
// beta2^t); update == 0 only rewrites the BF16 weight copies.
struct MlpAdam {
    int update;
    float lr, beta1, beta2, eps, c1, c2;
};
// Weight and bias gradients from the stored signals (after a training
// forward of the same B) into d.grad, and the loss into *loss (may be
// null); with adam (may be null) also the Adam step of every parameter and
// its BF16 copies, as each gradient tile completes.
hipError_t launch_mlp_wgrad(const MlpDev& d, int B, float* loss, hipStream_t s, const MlpAdam* adam = nullptr);
// Adam on d.grad (a.update != 0), then the BF16 weight copies.
hipError_t launch_mlp_adam(const MlpDev& d, const MlpAdam& a, hipStream_t s);
// Features of n states into X [n][21]; with U and Y also the normalised
// targets Y [n][126] = U [n][u_stride] / tau_max.
hipError_t launch_mlp_features(const MlpDev& d, int n, const double* q, const double* qd, const double* target,
                               float* X, const double* U, int u_stride, float* Y, hipStream_t s);

}  // namespace mppi
