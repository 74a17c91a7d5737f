// mlp.hip -- the proposal network on gfx950: BF16 matrix-core products
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation.
//
//   mlp_forward_kernel<TRAIN>  one workgroup (16 waves, each holding 16 of a
//                   layer's output columns) per 16 states (one
//                   matrix-core row tile, so a 512-row batch spreads over 32
//                   workgroups); the layers run back to back with the
//                   activation tile in LDS; each layer's weight fragments
//                   are requested one layer ahead.  A proposal encodes the
//                   input features from the states in the same launch (one
//                   launch per proposal).  Training adds the MSE signal and the backward
//                   products e_{l-1} = (e_l W_l) * gelu'(z_{l-1}) in the same
//                   workgroup (the rows are independent; the
//                   pre-activations stay in registers), storing every
//                   activation and signal transposed for the weight gradients.
//   mlp_wgrad_kernel   dW_l = e_l^T a_{l-1} (a contraction over the batch),
//                   one workgroup per 32 x 32 tile of one layer, its 16
//                   waves splitting the batch; db_l = sum of e_l.
//   mlp_adam_kernel    Adam on the FP32 master weights, then the BF16 copies
//                   (row-major and transposed); a training step applies the
//                   same update in mlp_wgrad_kernel as each tile completes.
//   mlp_features_kernel  (q/q_max, qd/qd_max, p_des, quat_des with w >= 0)
//                   of recorded states for training rows, and optionally
//                   the normalised targets U* / tau_max.
//
// Matrix-core fragments (16 x 16 x 32): lane l holds row (l mod 16) of A
// and column (l mod 16) of B with the k values 8 (l div 16) + 0..7 of the
// step, one 16-byte read per operand; the FP32 result holds column
// (l mod 16), rows 4 (l div 16) + 0..3.  Every operand is read with k
// contiguous: A from the LDS tile [row][k] (row stride 264 BF16: the 16
// rows of a lane group start on distinct banks), B^T from the weights
// [n][k] (forward) or from their stored transposes (backward), both
// operands of the weight gradient from the transposed [feature][batch]
// buffers; the global ones are kept in operand order (frag_index), one
// contiguous 1 KB read per fragment.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "mlp.hpp"

namespace mppi {
namespace {

typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kFwdWaves = 16;                         // waves of a forward workgroup
constexpr int kThreads = 64 * kFwdWaves;
constexpr int kHidCT = kMlpHid / 16 / kFwdWaves;      // column tiles per wave: hidden layers
// the output layer's 8 column tiles go to its first kOutWaves waves
constexpr int kOutWaves = kMlpOutPad / 16 < kFwdWaves ? kMlpOutPad / 16 : kFwdWaves;
constexpr int kOutCT = kMlpOutPad / 16 / kOutWaves;
constexpr int kLda = 264;

// FP32 -> BF16, round to nearest, ties to even (NaN stays NaN)
__device__ __forceinline__ uint16_t to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// tanh(u) = 1 - 2 / (exp(2u) + 1) with the hardware exponential and
// reciprocal (absolute error ~1e-7, far below the BF16 rounding that
// follows; exp overflow gives the limits +-1 exactly)
__device__ __forceinline__ float tanh_fast(float u)
{
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * u) + 1.0f);
}

// tanh form of GELU and its derivative
__device__ __forceinline__ float gelu_f(float z)
{
    const float c = 0.7978845608028654f, a = 0.044715f;
    return 0.5f * z * (1.0f + tanh_fast(c * (z + a * z * z * z)));
}
__device__ __forceinline__ float gelu_d(float z)
{
    const float c = 0.7978845608028654f, a = 0.044715f;
    const float t = tanh_fast(c * (z + a * z * z * z));
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * c * (1.0f + 3.0f * a * z * z);
}

// 16 x 16 x 32: lane l holds row (l mod 16) of A and column (l mod 16) of
// B, each with the eight k values 8 (l div 16) + 0..7
__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                   0, 0);
}

constexpr int kRT = kMlpWgRows / 16;   // row tiles per workgroup

// Matrix-core operand order of a BF16 matrix [N][K] read as k-contiguous
// 16 x 32 fragments (the weights, their transposes, and the transposed
// activations and signals [feature][batch]): element (n, k) sits at
// ((n div 16) (K / 32) + k div 32) 512 + (n mod 16 + 16 ((k mod 32) div 8)) 8
// + k mod 8, so the fragment of column tile n div 16 and k-step k div 32 is
// 1 KB contiguous and lane l reads its 16 bytes at 16 l (a row-major layout
// spreads the same fragment over 16 half-used cache lines, which measured
// 2.3 times slower to fetch).  K is a multiple of 32.
__device__ __forceinline__ size_t frag_index(int n, int k, int K)
{
    return ((size_t)(n >> 4) * (K >> 5) + (k >> 5)) * 512 + ((n & 15) + 16 * ((k & 31) >> 3)) * 8 + (k & 7);
}

// The B fragments of one layer product held by one wave: CT column tiles
// from output column nb of Bt [N][K] in operand order (frag_index), in
// k-steps of 32 (16 x 16 x 32 products); each fragment is one contiguous
// 1 KB read.  The kernels request a layer's fragments one layer ahead, so
// their memory latency overlaps the previous layer's products.
template <int K, int CT> struct BFrag {
    static_assert(K % 32 == 0, "the contraction runs in chunks of 32");
    v8s b[K / 32][CT];
};
template <int K, int CT>
__device__ __forceinline__ void load_frag(const uint16_t* __restrict__ Bt, int nb, BFrag<K, CT>& f, int lane)
{
#pragma unroll
    for (int t = 0; t < K / 32; ++t)
#pragma unroll
        for (int j = 0; j < CT; ++j)
            f.b[t][j] = *reinterpret_cast<const v8s*>(Bt + ((size_t)((nb >> 4) + j) * (K / 32) + t) * 512 + lane * 8);
    // issue the loads here, not next to their products
    __builtin_amdgcn_sched_barrier(0);
}
// acc[i][j] = sum_k A[16 i + r][k] B[16 j + c][k] over the RT row tiles of
// the LDS tile A and the CT column tiles of f
template <int K, int CT>
__device__ __forceinline__ void frag_mm(const uint16_t* A, const BFrag<K, CT>& f, v4f (&acc)[kRT][CT], int lane)
{
    const int r = lane & 15, kg = (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < kRT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < K / 32; ++t) {
        v8s a[kRT];
#pragma unroll
        for (int i = 0; i < kRT; ++i) a[i] = *reinterpret_cast<const v8s*>(A + (16 * i + r) * kLda + 32 * t + kg);
#pragma unroll
        for (int i = 0; i < kRT; ++i)
#pragma unroll
            for (int j = 0; j < CT; ++j) acc[i][j] = mfma32(a[i], f.b[t][j], acc[i][j]);
    }
}

// LDS tile columns [0, ncols) -> global [c][Bp] at rows b0..b0+15 (the
// input tile only; the layers' outputs go out from their result registers)
__device__ __forceinline__ void store_transposed(const uint16_t* tile, int ncols, uint16_t* dst, int Bp, int b0,
                                                 int tid)
{
    for (int i = tid; i < ncols * kMlpWgRows; i += kThreads) {
        const int c = i / kMlpWgRows, r = i % kMlpWgRows;
        dst[frag_index(c, b0 + r, Bp)] = tile[r * kLda + c];
    }
}

// One result fragment's four BF16 values (column col, rows row0 + 0..3 of
// the workgroup's 16, row0 a multiple of 4) into the transposed global
// buffer [feature][Bp] in operand order: the four rows are contiguous there,
// so one 8-byte store per lane.
__device__ __forceinline__ void store_frag_T(uint16_t* dstT, int Bp, int b0, int row0, int col, const uint16_t (&o)[4])
{
    uint2 v;
    v.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
    v.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
    *reinterpret_cast<uint2*>(dstT + frag_index(col, b0 + row0, Bp)) = v;
}

// this wave's bias values of a hidden layer (columns nb + 16 j + lane mod 16)
__device__ __forceinline__ void load_bias(const float* __restrict__ bias, int nb, float (&bv)[kHidCT], int lane)
{
#pragma unroll
    for (int j = 0; j < kHidCT; ++j) bv[j] = bias[nb + 16 * j + (lane & 15)];
}

// hidden layer forward: out = bf16(gelu(A W^T + b)) from the wave's
// fragments f of W and bias values bv; the pre-activations go to zo (kept
// in registers for the backward pass, which needs exactly the values each
// thread computed here).  Rows past `rows` (padding of the last workgroup)
// are set to zero without evaluating GELU (rows never mix, so they cannot
// reach a valid output).
// Training (dstT non-null) also stores the activations transposed from the
// result registers (store_frag_T).
template <int K>
__device__ __forceinline__ void hidden_forward(const uint16_t* A, const BFrag<K, kHidCT>& f, const float (&bv)[kHidCT],
                                               float (&zo)[kRT][kHidCT][4], uint16_t* out, int rows, int w,
                                               int lane, uint16_t* dstT, int Bp, int b0)
{
    constexpr int NC = 16 * kHidCT;
    v4f acc[kRT][kHidCT];
    frag_mm(A, f, acc, lane);
#pragma unroll
    for (int i = 0; i < kRT; ++i)
#pragma unroll
        for (int j = 0; j < kHidCT; ++j) {
            const int col = w * NC + 16 * j + (lane & 15);
            uint16_t o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * i + 4 * (lane >> 4) + e;
                const float zz = acc[i][j][e] + bv[j];
                zo[i][j][e] = zz;
                // 16 i + e is the wave's smallest row of this element: past
                // `rows` no lane evaluates GELU (a uniform branch)
                o[e] = 0;
                if (16 * i + e < rows) o[e] = row < rows ? to_bf16(gelu_f(zz)) : (uint16_t)0;
                out[row * kLda + col] = o[e];
            }
            if (dstT) store_frag_T(dstT, Bp, b0, 16 * i + 4 * (lane >> 4), col, o);
        }
}

// hidden layer backward: bf16((E Wt^T) * gelu'(z)) from the wave's
// fragments f of Wt and the pre-activations zv this thread computed in the
// forward pass (same fragment map), into the LDS tile out (null for the
// first layer's signal, which no later product reads) and, transposed,
// into dstT
template <int K>
__device__ __forceinline__ void hidden_backward(const uint16_t* E, const BFrag<K, kHidCT>& f,
                                                const float (&zv)[kRT][kHidCT][4], uint16_t* out, int w, int lane,
                                                uint16_t* dstT, int Bp, int b0)
{
    constexpr int NC = 16 * kHidCT;
    v4f acc[kRT][kHidCT];
    frag_mm(E, f, acc, lane);
#pragma unroll
    for (int i = 0; i < kRT; ++i)
#pragma unroll
        for (int j = 0; j < kHidCT; ++j) {
            const int col = w * NC + 16 * j + (lane & 15);
            uint16_t o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * i + 4 * (lane >> 4) + e;
                o[e] = to_bf16(acc[i][j][e] * gelu_d(zv[i][j][e]));
                if (out) out[row * kLda + col] = o[e];
            }
            store_frag_T(dstT, Bp, b0, 16 * i + 4 * (lane >> 4), col, o);
        }
}

// Feature c (0..20) of state p: q / q_max, qd / qd_max, p_des, then the
// unit target quaternion with w >= 0 (the proposal's input encoding), in
// two halves: feature_load issues the loads, feature_value forms the value
// once they have arrived (so a kernel can request other operands between).
struct FeatIn {
    double v, s, qw, qx, qy, qz;
};
__device__ __forceinline__ FeatIn feature_load(const MlpDev& d, const double* __restrict__ q,
                                               const double* __restrict__ qd, const double* __restrict__ target,
                                               int p, int c)
{
    // every load unconditional (a select of the address), so that no
    // branch has to wait for them
    const double* tg = target + (size_t)p * 13;
    const double* src = c < 7 ? q + p * 7 + c : (c < 14 ? qd + p * 7 + (c - 7) : tg + (c - 14));
    FeatIn f;
    f.v = *src;
    f.s = d.scale[c < 14 ? c : 0];
    f.qw = tg[3]; f.qx = tg[4]; f.qy = tg[5]; f.qz = tg[6];
    return f;
}
__device__ __forceinline__ float feature_value(const FeatIn& f, int c)
{
    if (c < 14) return (float)(f.v / f.s);
    if (c < 17) return (float)f.v;
    const double nrm = sqrt(f.qw * f.qw + f.qx * f.qx + f.qy * f.qy + f.qz * f.qz);
    const double sg = (f.qw < 0.0 ? -1.0 : 1.0) / nrm;
    return (float)(f.v * sg);
}

template <bool TRAIN>
__global__ __launch_bounds__(kThreads) void mlp_forward_kernel(MlpDev d, const float* __restrict__ X, int B,
                                                               const float* __restrict__ Ytgt, float* __restrict__ Y,
                                                               double* __restrict__ U, int u_stride, float gscale,
                                                               const double* __restrict__ sq,
                                                               const double* __restrict__ sqd,
                                                               const double* __restrict__ stg)
{
    __shared__ __align__(16) uint16_t buf[2][kMlpWgRows * kLda];
    __shared__ float red[kThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int b0 = blockIdx.x * kMlpWgRows;
    const float* th = d.theta;

    const int nh = w * 16 * kHidCT;   // this wave's first column of a hidden layer
    // a_0 = bf16(x), x from X or (X null) encoded here from the states
    // (one element per thread; feature columns 21..31 and rows past B are
    // zero): its loads first, then the first two layers' operands, and only
    // then the input tile's values (the loads return in order)
    static_assert(kMlpWgRows * kMlpInPad <= kThreads, "one input element per thread");
    const int ir = tid / kMlpInPad, ic = tid % kMlpInPad;
    const bool has_x = tid < kMlpWgRows * kMlpInPad && ic < kMlpIn && b0 + ir < B;
    // the element's indices clamped to a valid one, so that the loads need
    // no branch (has_x decides below whether the value is used)
    const int pr = min(b0 + ir, B - 1), pc = min(ic, kMlpIn - 1);
    float xv = 0.0f;
    FeatIn fin{0.0, 1.0, 0.0, 0.0, 0.0, 0.0};
    if (TRAIN || X) xv = X[(size_t)pr * kMlpIn + pc];   // training always has X
    else fin = feature_load(d, sq, sqd, stg, pr, pc);
    __builtin_amdgcn_sched_barrier(0);
    BFrag<kMlpInPad, kHidCT> f1;
    BFrag<kMlpHid, kHidCT> f2;
    float bv1[kHidCT], bv2[kHidCT];
    load_frag(d.W1, nh, f1, lane);
    load_bias(th + kOffB1, nh, bv1, lane);
    load_frag(d.W2, nh, f2, lane);
    load_bias(th + kOffB2, nh, bv2, lane);
    __builtin_amdgcn_sched_barrier(0);
    if (tid < kMlpWgRows * kMlpInPad) {
        float x = 0.0f;
        if (has_x) x = (TRAIN || X) ? xv : feature_value(fin, pc);
        buf[0][ir * kLda + ic] = to_bf16(x);
    }
    __syncthreads();
    if (TRAIN) store_transposed(buf[0], kMlpInPad, d.aT0, d.Bp, b0, tid);

    // training keeps every row (the backward pass reads them all)
    const int rows = TRAIN ? kMlpWgRows : min(kMlpWgRows, B - b0);
    float z1[kRT][kHidCT][4], z2[kRT][kHidCT][4], z3[kRT][kHidCT][4];
    hidden_forward<kMlpInPad>(buf[0], f1, bv1, z1, buf[1], rows, w, lane, TRAIN ? d.aT1 : nullptr, d.Bp, b0);
    __syncthreads();
    BFrag<kMlpHid, kHidCT> f3;
    float bv3[kHidCT];
    load_frag(d.W3, nh, f3, lane);
    load_bias(th + kOffB3, nh, bv3, lane);
    hidden_forward<kMlpHid>(buf[1], f2, bv2, z2, buf[0], rows, w, lane, TRAIN ? d.aT2 : nullptr, d.Bp, b0);
    __syncthreads();

    // the output layer's operands (its 8 column tiles on the first waves)
    constexpr int NO = 16 * kOutCT;
    BFrag<kMlpHid, kOutCT> f4;
    float b4[kOutCT], yt[kRT][kOutCT][4];
    double us[kOutCT];   // inference into U: the torque limit of the column's joint
    if (w < kOutWaves) {
        load_frag(d.W4, w * NO, f4, lane);
#pragma unroll
        for (int j = 0; j < kOutCT; ++j) {
            const int col = w * NO + 16 * j + (lane & 15);
            b4[j] = col < kMlpOut ? th[kOffB4 + col] : 0.0f;
            us[j] = (!TRAIN && U) ? d.scale[14 + col % 7] : 0.0;
#pragma unroll
            for (int i = 0; i < kRT; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 16 * i + 4 * (lane >> 4) + e;
                    yt[i][j][e] = (TRAIN && col < kMlpOut && b0 + row < B) ? Ytgt[(size_t)(b0 + row) * kMlpOut + col]
                                                                          : 0.0f;
                }
        }
    }
    hidden_forward<kMlpHid>(buf[0], f3, bv3, z3, buf[1], rows, w, lane, TRAIN ? d.aT3 : nullptr, d.Bp, b0);
    __syncthreads();

    // output layer; training: e_4 = bf16(2 (y - y*) / (B 126)) into buf[0]
    BFrag<kMlpOutPad, kHidCT> g4;
    {
        float sq = 0.0f;
        if (w < kOutWaves) {
            v4f acc[kRT][kOutCT];
            frag_mm(buf[1], f4, acc, lane);
#pragma unroll
            for (int i = 0; i < kRT; ++i)
#pragma unroll
                for (int j = 0; j < kOutCT; ++j) {
                    const int col = w * NO + 16 * j + (lane & 15);
                    uint16_t o[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = 16 * i + 4 * (lane >> 4) + e;
                        const bool valid = col < kMlpOut && b0 + row < B;
                        const float y = acc[i][j][e] + b4[j];
                        if (!TRAIN && valid) {   // training writes neither
                            if (Y) Y[(size_t)(b0 + row) * kMlpOut + col] = y;
                            if (U) U[(size_t)(b0 + row) * u_stride + col] = us[j] * (double)y;
                        }
                        if (TRAIN) {
                            const float res = valid ? y - yt[i][j][e] : 0.0f;
                            sq += res * res;
                            o[e] = to_bf16(res * gscale);
                            buf[0][row * kLda + col] = o[e];
                        }
                    }
                    if (TRAIN) store_frag_T(d.eT4, d.Bp, b0, 16 * i + 4 * (lane >> 4), col, o);
                }
        }
        if (!TRAIN) return;
        load_frag(d.W4t, nh, g4, lane);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
        if (lane == 0) red[w] = sq;
    }
    __syncthreads();
    if (tid == 0) {
        float sl = 0.0f;
#pragma unroll
        for (int q = 0; q < kFwdWaves; ++q) sl += red[q];
        d.lossp[blockIdx.x] = sl;
    }

    BFrag<kMlpHid, kHidCT> g3;
    load_frag(d.W3t, nh, g3, lane);
    hidden_backward<kMlpOutPad>(buf[0], g4, z3, buf[1], w, lane, d.eT3, d.Bp, b0);
    __syncthreads();
    BFrag<kMlpHid, kHidCT> g2;
    load_frag(d.W2t, nh, g2, lane);
    hidden_backward<kMlpHid>(buf[1], g3, z2, buf[0], w, lane, d.eT2, d.Bp, b0);
    __syncthreads();
    hidden_backward<kMlpHid>(buf[0], g2, z1, nullptr, w, lane, d.eT1, d.Bp, b0);
}

// Adam state of one parameter, read before its gradient is known
struct AdamState {
    float th, m, v;
};
__device__ __forceinline__ AdamState adam_load(const MlpDev& d, int i, const MlpAdam& a)
{
    AdamState s{d.theta[i], 0.0f, 0.0f};
    if (a.update) {
        s.m = d.m[i];
        s.v = d.v[i];
    }
    return s;
}

// Adam step of parameter i with gradient g (a.update != 0) from its state
// s, then its BF16 copies: W row-major and, for layers 2-4, the transposes.
// No multiply-add contraction, so that the fused step in the
// weight-gradient launch and the separate Adam launch round alike.
__device__ __forceinline__ void adam_apply(const MlpDev& d, int i, float g, const MlpAdam& a, AdamState s)
{
#pragma clang fp contract(off)
    float th = s.th;
    if (a.update) {
        const float m = a.beta1 * s.m + (1.0f - a.beta1) * g;
        const float v = a.beta2 * s.v + (1.0f - a.beta2) * g * g;
        th -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
        d.m[i] = m;
        d.v[i] = v;
        d.theta[i] = th;
    }
    const uint16_t h = to_bf16(th);
    if (i < kOffB1) {
        const int n = i / kMlpIn, k = i % kMlpIn;
        d.W1[frag_index(n, k, kMlpInPad)] = h;
    } else if (i >= kOffW2 && i < kOffB2) {
        const int j = i - kOffW2, n = j / kMlpHid, k = j % kMlpHid;
        d.W2[frag_index(n, k, kMlpHid)] = h;
        d.W2t[frag_index(k, n, kMlpHid)] = h;
    } else if (i >= kOffW3 && i < kOffB3) {
        const int j = i - kOffW3, n = j / kMlpHid, k = j % kMlpHid;
        d.W3[frag_index(n, k, kMlpHid)] = h;
        d.W3t[frag_index(k, n, kMlpHid)] = h;
    } else if (i >= kOffW4 && i < kOffB4) {
        const int j = i - kOffW4, n = j / kMlpHid, k = j % kMlpHid;
        d.W4[frag_index(n, k, kMlpHid)] = h;
        d.W4t[frag_index(k, n, kMlpOutPad)] = h;
    }
}

// Weight and bias gradients dW_l = e_l^T a_{l-1}, db_l = e_l^T 1 (a
// contraction over the batch).  Tiles of 32 x 32 of the gradient matrices:
// layer 1 8 (256 x 32 padded), layers 2, 3 64 each, layer 4 32 (128 padded
// x 256).  A workgroup takes one tile; its 16 waves split the batch (in
// k-steps of 32 rows, kWgradChunk requested together), so that a CU has
// sixteen waves' loads in flight, and add their partial tiles in LDS, in
// wave order.  The tiles of the first column also form the bias gradients
// on the matrix cores, from the same e fragments times a fragment of ones
// (every column of that product is db).  Every thread then finishes one
// element of the tile: the gradient and, fused, its Adam step, whose state
// it requested at the start (that latency overlaps the contraction).
constexpr int kWgradTiles = 8 + 64 + 64 + 32;
constexpr int kWgradWaves = 16;
constexpr int kWgradChunk = 4;    // k-steps of 32 rows requested together

__global__ __launch_bounds__(64 * kWgradWaves) void mlp_wgrad_kernel(MlpDev d, int B, float* loss, int fuse,
                                                                     MlpAdam adam)
{
    static_assert(64 * kWgradWaves == 32 * 32, "one thread per element of a tile");
    __shared__ float part[kWgradWaves][32 * 32];
    __shared__ float bpart[kWgradWaves][32];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // Tile of this workgroup.  Workgroup b runs on XCD b mod 8 and every
    // layer's range starts at a multiple of 8, so within a layer x = t mod
    // 8 is the XCD: the tiles of a layer are laid out 2 x 4 over the XCDs
    // (a layer of 8 x 8 tiles gives each XCD 4 row blocks of E by 2 of the
    // activations, the 4 x 8 layer 2 x 2), so that an XCD's L2 fetches
    // half of E and a quarter of the activations instead of all of one.
    int t = blockIdx.x;
    const uint16_t *E, *Act;
    int nreal, kreal, woff, boff, tm, tn;
    auto place = [&](int tt, int rows_per) {   // rows_per: row blocks of E per XCD row
        const int x = tt % 8, slot = tt / 8;
        tm = (x / 4) * rows_per + slot / 2;
        tn = (x % 4) * 2 + slot % 2;
    };
    if (t < 8) {
        E = d.eT1; Act = d.aT0; nreal = kMlpHid; kreal = kMlpIn; woff = kOffW1; boff = kOffB1; tm = t; tn = 0;
    } else if (t < 72) {
        E = d.eT2; Act = d.aT1; nreal = kMlpHid; kreal = kMlpHid; woff = kOffW2; boff = kOffB2;
        place(t - 8, 4);
    } else if (t < 136) {
        E = d.eT3; Act = d.aT2; nreal = kMlpHid; kreal = kMlpHid; woff = kOffW3; boff = kOffB3;
        place(t - 72, 4);
    } else {
        E = d.eT4; Act = d.aT3; nreal = kMlpOut; kreal = kMlpHid; woff = kOffW4; boff = kOffB4;
        place(t - 136, 2);
    }
    const int m0 = tm * 32, n0 = tn * 32, Bp = d.Bp;
    const bool bias = tn == 0;
    // the element this thread finishes (row rl, column cl of the tile) and,
    // on bias tiles, threads 0..31 also bias m0 + tid: their Adam state now
    const int rl = tid >> 5, cl = tid & 31;
    const bool own = m0 + rl < nreal && n0 + cl < kreal;
    const int pw = woff + (m0 + rl) * kreal + n0 + cl;
    const bool ownb = bias && tid < 32 && m0 + tid < nreal;
    const int pb = boff + m0 + tid;
    AdamState sw{0.0f, 0.0f, 0.0f}, sb{0.0f, 0.0f, 0.0f};
    if (fuse && own) sw = adam_load(d, pw, adam);
    if (fuse && ownb) sb = adam_load(d, pb, adam);

    // rows of this batch: the forward workgroups covered ceil(B / 64) * 64
    // (rows past B carry e = 0); later rows of the buffers are stale.  This
    // wave's k-steps of 32 rows: [s0, s1) of Bb / 32
    const int nb = (B + kMlpRows - 1) / kMlpRows, Bb = nb * kMlpRows;
    const int P = Bb / 32, per = (P + kWgradWaves - 1) / kWgradWaves;
    const int s0 = min(P, w * per), s1 = min(P, s0 + per);
    // operand order (frag_index): row tile m, k-step s at (m (Bp / 32) + s) 512
    const int r = lane & 15;
    const size_t ts = (size_t)(Bp / 32) * 512;
    const uint16_t* ea[2] = {E + (size_t)(m0 >> 4) * ts + lane * 8, E + (size_t)((m0 >> 4) + 1) * ts + lane * 8};
    const uint16_t* ab[2] = {Act + (size_t)(n0 >> 4) * ts + lane * 8, Act + (size_t)((n0 >> 4) + 1) * ts + lane * 8};
    v4f acc[2][2], accb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        accb[i] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    }
    const short one = 0x3f80;   // BF16 1.0
    const v8s ones = {one, one, one, one, one, one, one, one};
    for (int st = s0; st < s1; st += kWgradChunk) {
        const int ns = min(kWgradChunk, s1 - st);
        v8s a[kWgradChunk][2], b[kWgradChunk][2];
#pragma unroll
        for (int q = 0; q < kWgradChunk; ++q)
            if (q < ns)
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    a[q][i] = *reinterpret_cast<const v8s*>(ea[i] + (size_t)(st + q) * 512);
                    b[q][i] = *reinterpret_cast<const v8s*>(ab[i] + (size_t)(st + q) * 512);
                }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < kWgradChunk; ++q)
            if (q < ns)
#pragma unroll
                for (int i = 0; i < 2; ++i) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) acc[i][j] = mfma32(a[q][i], b[q][j], acc[i][j]);
                    if (bias) accb[i] = mfma32(a[q][i], ones, accb[i]);
                }
    }
    // every wave's partial tile (and db column) into LDS; then every
    // thread sums its element over the waves in wave order
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) part[w][(16 * i + 4 * (lane >> 4) + e) * 32 + 16 * j + r] = acc[i][j][e];
    // column 0 of the db product: rows 16 i + 4 (lane div 16) + e
    if (bias && r == 0)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) bpart[w][16 * i + 4 * (lane >> 4) + e] = accb[i][e];
    __syncthreads();
    if (own) {
        float v = part[0][tid];
#pragma unroll
        for (int q = 1; q < kWgradWaves; ++q) v += part[q][tid];
        d.grad[pw] = v;
        if (fuse) adam_apply(d, pw, v, adam, sw);
    }
    if (ownb) {
        float v = bpart[0][tid];
#pragma unroll
        for (int q = 1; q < kWgradWaves; ++q) v += bpart[q][tid];
        d.grad[pb] = v;
        if (fuse) adam_apply(d, pb, v, adam, sb);
    }
    // the loss: the forward workgroups' sums reduced by workgroup 0 (every
    // thread a strided share, then the waves' shuffles and LDS), not by one
    // thread's chain of dependent loads
    if (blockIdx.x == 0 && loss) {
        __shared__ float lred[kWgradWaves];
        float sl = 0.0f;
        for (int i = tid; i < Bb / kMlpWgRows; i += 64 * kWgradWaves) sl += d.lossp[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sl += __shfl_xor(sl, o);
        if (lane == 0) lred[w] = sl;
        __syncthreads();
        if (tid == 0) {
            float tot = 0.0f;
#pragma unroll
            for (int q = 0; q < kWgradWaves; ++q) tot += lred[q];
            *loss = tot / ((float)B * (float)kMlpOut);
        }
    }
}

__global__ void mlp_adam_kernel(MlpDev d, MlpAdam a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpParams) return;
    adam_apply(d, i, a.update ? d.grad[i] : 0.0f, a, adam_load(d, i, a));
}

__global__ void mlp_features_kernel(MlpDev d, int n, const double* __restrict__ q, const double* __restrict__ qd,
                                    const double* __restrict__ target, float* __restrict__ X,
                                    const double* __restrict__ U, int u_stride, float* __restrict__ Y)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (U && Y)   // normalised training targets y* = U* / tau_max
        for (int c = 0; c < kMlpOut; ++c) Y[(size_t)p * kMlpOut + c] = (float)(U[(size_t)p * u_stride + c] / d.scale[14 + c % 7]);
    float* x = X + (size_t)p * kMlpIn;
    for (int c = 0; c < kMlpIn; ++c) x[c] = feature_value(feature_load(d, q, qd, target, p, c), c);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t mlp_scratch_bytes(int Bp)
{
    const size_t P = kMlpParams;
    size_t b = 0;
    b += 4 * align256(P * sizeof(float));                                      // theta, m, v, grad
    b += align256((size_t)kMlpHid * kMlpInPad * 2) + 2 * align256((size_t)kMlpHid * kMlpHid * 2) +
         align256((size_t)kMlpOutPad * kMlpHid * 2);                           // W1..W4
    b += 2 * align256((size_t)kMlpHid * kMlpHid * 2) + align256((size_t)kMlpHid * kMlpOutPad * 2);   // W2t..W4t
    b += align256((size_t)kMlpInPad * Bp * 2) + 3 * align256((size_t)kMlpHid * Bp * 2);   // aT0..aT3
    b += 3 * align256((size_t)kMlpHid * Bp * 2) + align256((size_t)kMlpOutPad * Bp * 2);  // eT1..eT4
    b += align256((size_t)(Bp / kMlpWgRows) * sizeof(float));                  // lossp
    b += align256(21 * sizeof(double));                                        // scale
    return b;
}

void mlp_carve(MlpDev& d, void* base, int Bp)
{
    char* p = static_cast<char*>(base);
    auto take = [&](size_t bytes) { char* q = p; p += align256(bytes); return q; };
    const size_t P = kMlpParams;
    d.theta = (float*)take(P * 4);
    d.m = (float*)take(P * 4);
    d.v = (float*)take(P * 4);
    d.grad = (float*)take(P * 4);
    d.W1 = (uint16_t*)take((size_t)kMlpHid * kMlpInPad * 2);
    d.W2 = (uint16_t*)take((size_t)kMlpHid * kMlpHid * 2);
    d.W3 = (uint16_t*)take((size_t)kMlpHid * kMlpHid * 2);
    d.W4 = (uint16_t*)take((size_t)kMlpOutPad * kMlpHid * 2);
    d.W2t = (uint16_t*)take((size_t)kMlpHid * kMlpHid * 2);
    d.W3t = (uint16_t*)take((size_t)kMlpHid * kMlpHid * 2);
    d.W4t = (uint16_t*)take((size_t)kMlpHid * kMlpOutPad * 2);
    d.aT0 = (uint16_t*)take((size_t)kMlpInPad * Bp * 2);
    d.aT1 = (uint16_t*)take((size_t)kMlpHid * Bp * 2);
    d.aT2 = (uint16_t*)take((size_t)kMlpHid * Bp * 2);
    d.aT3 = (uint16_t*)take((size_t)kMlpHid * Bp * 2);
    d.eT1 = (uint16_t*)take((size_t)kMlpHid * Bp * 2);
    d.eT2 = (uint16_t*)take((size_t)kMlpHid * Bp * 2);
    d.eT3 = (uint16_t*)take((size_t)kMlpHid * Bp * 2);
    d.eT4 = (uint16_t*)take((size_t)kMlpOutPad * Bp * 2);
    d.lossp = (float*)take((size_t)(Bp / kMlpWgRows) * 4);
    d.scale = (const double*)take(21 * sizeof(double));
    d.Bp = Bp;
}

hipError_t launch_mlp_forward(const MlpDev& d, const float* X, int B, const float* Ytgt, float* Y, double* U,
                              int u_stride, hipStream_t s, const double* q, const double* qd, const double* target)
{
    if (B < 1 || B > d.Bp || (!X && (Ytgt || !q || !qd || !target))) return hipErrorInvalidValue;
    const float gscale = 2.0f / ((float)B * (float)kMlpOut);
    if (Ytgt) {
        // training covers the batch rounded up to 64 rows (padding rows carry
        // zero inputs and zero signals; the weight gradients split that range)
        const dim3 grid((B + kMlpRows - 1) / kMlpRows * (kMlpRows / kMlpWgRows));
        hipLaunchKernelGGL(mlp_forward_kernel<true>, grid, dim3(kThreads), 0, s, d, X, B, Ytgt, Y, U, u_stride, gscale,
                           q, qd, target);
    } else {
        const dim3 grid((B + kMlpWgRows - 1) / kMlpWgRows);
        hipLaunchKernelGGL(mlp_forward_kernel<false>, grid, dim3(kThreads), 0, s, d, X, B, Ytgt, Y, U, u_stride,
                           gscale, q, qd, target);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_wgrad(const MlpDev& d, int B, float* loss, hipStream_t s, const MlpAdam* adam)
{
    if (B < 1 || B > d.Bp) return hipErrorInvalidValue;
    const MlpAdam a = adam ? *adam : MlpAdam{0, 0.f, 0.f, 0.f, 1.f, 1.f, 1.f};
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3(kWgradTiles), dim3(64 * kWgradWaves), 0, s, d, B, loss,
                       adam ? 1 : 0, a);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(const MlpDev& d, const MlpAdam& a, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, d, a);
    return hipGetLastError();
}

hipError_t launch_mlp_features(const MlpDev& d, int n, const double* q, const double* qd, const double* target,
                               float* X, const double* U, int u_stride, float* Y, hipStream_t s)
{
    if (n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mlp_features_kernel, dim3((n + 63) / 64), dim3(64), 0, s, d, n, q, qd, target, X, U,
                       u_stride, Y);
    return hipGetLastError();
}

}  // namespace mppi
