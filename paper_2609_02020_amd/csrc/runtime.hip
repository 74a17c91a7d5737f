// runtime.hip -- the C ABI of libmppi.so (include/mppi.h): handle
// lifecycle, argument validation, device buffers and launch sequencing.
// All arithmetic of the method runs in the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unistd.h>

#include "launch.hpp"
#include "model_prep.hpp"
#include "mppi.h"

using namespace mppi;

struct mppi_solver {
    mppi_robot_params robot;
    mppi_cost_params cost;
    int device = 0;
    mppi_robot_params* d_raw = nullptr;
    ModelM<float>* d_mf = nullptr;
    ModelM<double>* d_md = nullptr;
    CostM<float>* d_cf = nullptr;
    CostM<double>* d_cd = nullptr;
    void* d_noise = nullptr;     // R [T][7][K]
    void* d_costs = nullptr;     // R [K]
    void* d_parts = nullptr;     // per-wave Eq. 4 partials (FP64-sized)
    unsigned int* d_counter = nullptr;  // last-block counter of the fused one-/two-wave updates
    int* d_status = nullptr;
    double* d_iter = nullptr;    // [2][T][7]: U of the intermediate iterations
    double* d_io = nullptr;      // q 7 | qd 7 | target 13 | U_nom T*7 | U_new T*7
    double* h_io = nullptr;      // pinned mirror of d_io
    void* h_costs = nullptr;     // pinned R [K]
    int* h_status = nullptr;     // pinned
    hipStream_t stream = nullptr;
    int waves_per_group = 8;     // mppi_set_launch
};

namespace {

constexpr int kIoQ = 0, kIoQd = 7, kIoTarget = 14, kIoU = 27;

size_t rsize(const mppi_cost_params& c) { return c.precision == MPPI_FP64 ? sizeof(double) : sizeof(float); }

bool finite_all(const double* p, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// Sylvester's criterion on a symmetric 3x3 given as xx yy zz xy xz yz.
bool sym3_pd(double xx, double yy, double zz, double xy, double xz, double yz, double tol)
{
    double m1 = xx, m2 = xx * yy - xy * xy;
    double m3 = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz);
    return m1 > tol && m2 > tol * tol && m3 > tol * tol * tol;
}

bool sym3_psd(double xx, double yy, double zz, double xy, double xz, double yz, double tol)
{
    // all principal minors >= -tol
    if (xx < -tol || yy < -tol || zz < -tol) return false;
    if (xx * yy - xy * xy < -tol || xx * zz - xz * xz < -tol || yy * zz - yz * yz < -tol) return false;
    double d = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz);
    return d >= -tol;
}

int validate_robot(const mppi_robot_params* r)
{
    if (!r || r->n_joints != MPPI_NJ) return MPPI_EINVAL;
    for (int i = 0; i < MPPI_NJ; ++i) {
        const mppi_link_params& L = r->link[i];
        if (!finite_all(L.R_parent, 9) || !finite_all(L.r_parent, 3) || !finite_all(L.com, 3) ||
            !finite_all(L.inertia_com, 6))
            return MPPI_EINVAL;
        double s[6] = {L.mass, L.armature, L.q_min, L.q_max, L.qd_max, L.tau_max};
        if (!finite_all(s, 6) || !(L.mass > 0) || L.armature < 0 || !(L.q_min < L.q_max) ||
            !(L.qd_max > 0) || !(L.tau_max > 0))
            return MPPI_EINVAL;
        const double* I = L.inertia_com;
        if (!sym3_pd(I[0], I[1], I[2], I[3], I[4], I[5], 0.0)) return MPPI_EINVAL;
        // triangle inequality <=> tr(I)/2 * 1 - I is positive semidefinite
        double h = 0.5 * (I[0] + I[1] + I[2]);
        double tol = 1e-12 * (1.0 + h);
        if (!sym3_psd(h - I[0], h - I[1], h - I[2], -I[3], -I[4], -I[5], tol)) return MPPI_EINVAL;
        // R_parent must be a rotation
        const double* R = L.R_parent;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double d = R[a * 3] * R[b * 3] + R[a * 3 + 1] * R[b * 3 + 1] + R[a * 3 + 2] * R[b * 3 + 2];
                if (std::fabs(d - (a == b ? 1.0 : 0.0)) > 1e-9) return MPPI_EINVAL;
            }
    }
    if (!finite_all(r->R_ee, 9) || !finite_all(r->r_ee, 3) || !finite_all(r->gravity, 3)) return MPPI_EINVAL;
    return MPPI_OK;
}

int validate_cost(const mppi_cost_params* c)
{
    if (!c) return MPPI_EINVAL;
    if (c->K < 1 || c->K > (1 << 20) || c->T < 1 || c->T > kMaxT) return MPPI_EINVAL;
    if (!(c->dt > 0) || !std::isfinite(c->dt) || !(c->lambda > 0) || !std::isfinite(c->lambda)) return MPPI_EINVAL;
    for (int j = 0; j < MPPI_NJ; ++j)
        if (!(c->sigma[j] >= 0) || !std::isfinite(c->sigma[j])) return MPPI_EINVAL;
    const double* groups[] = {c->W_pos, c->W_ori, c->W_force, c->W_reg, c->q_rest, c->F_ext, c->wall_n};
    const int sizes[] = {3, 3, 6, 6, MPPI_NJ, 6, 3};
    for (int g = 0; g < 7; ++g)
        if (!finite_all(groups[g], sizes[g])) return MPPI_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (c->W_pos[a] < 0 || c->W_ori[a] < 0) return MPPI_EINVAL;
    for (int a = 0; a < 6; ++a)
        if (c->W_force[a] < 0 || c->W_reg[a] < 0) return MPPI_EINVAL;
    double s[] = {c->w_q, c->w_qd, c->w_tau, c->w_post, c->w_terminal, c->wall_d0, c->wall_k, c->wall_c,
                  c->lambda_fp64_threshold};
    if (!finite_all(s, 9)) return MPPI_EINVAL;
    if (c->w_q < 0 || c->w_qd < 0 || c->w_tau < 0 || c->w_post < 0 || c->w_terminal < 0) return MPPI_EINVAL;
    if (c->force_mode != 0 && c->force_mode != 1) return MPPI_EINVAL;
    if (c->ext_mode < MPPI_EXT_NONE || c->ext_mode > MPPI_EXT_WALL) return MPPI_EINVAL;
    if (c->precision != MPPI_FP32 && c->precision != MPPI_FP64) return MPPI_EINVAL;
    if (c->ext_mode == MPPI_EXT_WALL) {
        double n = std::sqrt(c->wall_n[0] * c->wall_n[0] + c->wall_n[1] * c->wall_n[1] + c->wall_n[2] * c->wall_n[2]);
        if (std::fabs(n - 1.0) > 1e-6 || c->wall_k < 0 || c->wall_c < 0) return MPPI_EINVAL;
    }
    if (c->dynamics != MPPI_DYN_ABA && c->dynamics != MPPI_DYN_EXPLICIT_M) return MPPI_EINVAL;
    // collision term
    if (!std::isfinite(c->w_collision) || c->w_collision < 0) return MPPI_EINVAL;
    if (c->n_obstacles < 0 || c->n_obstacles > MPPI_MAX_OBSTACLES) return MPPI_EINVAL;
    if (c->n_pairs < 0 || c->n_pairs > MPPI_MAX_PAIRS) return MPPI_EINVAL;
    for (int o = 0; o < c->n_obstacles; ++o)
        if (!finite_all(c->obstacles[o], 6)) return MPPI_EINVAL;
    for (int i = 0; i < c->n_pairs; ++i) {
        const int nseg = MPPI_NJ + c->n_obstacles;
        if (c->pairs[i][0] < 0 || c->pairs[i][0] >= nseg || c->pairs[i][1] < 0 || c->pairs[i][1] >= nseg)
            return MPPI_EINVAL;
        if (!std::isfinite(c->d_th[i]) || c->d_th[i] < 0) return MPPI_EINVAL;
    }
    if (!(c->noise_rho >= 0.0 && c->noise_rho < 1.0)) return MPPI_EINVAL;
    if (c->iterations < 0 || c->iterations > MPPI_MAX_ITERATIONS) return MPPI_EINVAL;
    return MPPI_OK;
}

int iterations_of(const mppi_cost_params& c) { return c.iterations > 1 ? c.iterations : 1; }

// do [a, a + n) and [b, b + n) (doubles) share an address?
bool ranges_overlap(const double* a, const double* b, size_t n)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    const uintptr_t len = n * sizeof(double);
    return x < y + len && y < x + len;
}

bool has_force(const mppi_cost_params& c)
{
    for (int a = 0; a < 6; ++a)
        if (c.W_force[a] != 0.0 || c.W_reg[a] != 0.0) return true;
    return false;
}

int upload_cost(mppi_solver* h)
{
    CostM<float> cf;
    CostM<double> cd;
    prep_cost(h->cost, cf);
    prep_cost(h->cost, cd);
    if (hipMemcpy(h->d_cf, &cf, sizeof cf, hipMemcpyHostToDevice) != hipSuccess) return MPPI_EDEVICE;
    if (hipMemcpy(h->d_cd, &cd, sizeof cd, hipMemcpyHostToDevice) != hipSuccess) return MPPI_EDEVICE;
    return MPPI_OK;
}

void release(mppi_solver* h)
{
    if (!h) return;
    (void)hipFree(h->d_raw);
    (void)hipFree(h->d_mf);
    (void)hipFree(h->d_md);
    (void)hipFree(h->d_cf);
    (void)hipFree(h->d_cd);
    (void)hipFree(h->d_noise);
    (void)hipFree(h->d_costs);
    (void)hipFree(h->d_parts);
    (void)hipFree(h->d_counter);
    (void)hipFree(h->d_status);
    (void)hipFree(h->d_iter);
    (void)hipFree(h->d_io);
    (void)hipHostFree(h->h_io);
    (void)hipHostFree(h->h_costs);
    (void)hipHostFree(h->h_status);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

bool acc64_of(const mppi_cost_params& c) { return c.precision == MPPI_FP64 || c.lambda < c.lambda_fp64_threshold; }

int update_enqueue_one(mppi_solver* h, const mppi_device_io* io, hipStream_t s, void* noise, void* costs,
                       bool merge, bool want_noise)
{
    UpdateArgs a;
    a.want_noise = want_noise ? 1 : 0;
    const bool fp64 = h->cost.precision == MPPI_FP64;
    a.model = fp64 ? (const void*)h->d_md : (const void*)h->d_mf;
    a.cost = fp64 ? (const void*)h->d_cd : (const void*)h->d_cf;
    a.q0 = io->q;
    a.qd0 = io->qd;
    a.target = io->target;
    a.U_nom = io->U_nominal;
    a.seed = io->seed;
    a.tick = io->tick;
    a.K = h->cost.K;
    a.T = h->cost.T;
    a.lambda = h->cost.lambda;
    a.noise = noise;
    a.costs = costs;
    a.merge = merge ? 1 : 0;
    a.parts = h->d_parts;
    a.counter = h->d_counter;
    a.U_new = io->U_new;
    a.U_shift = io->U_shift;
    a.status = io->status;
    a.dynamics = h->cost.dynamics;
    a.collision = h->cost.n_pairs > 0 ? 1 : 0;
    a.waves_per_group = h->waves_per_group;
    return launch_update(h->cost.precision, acc64_of(h->cost), has_force(h->cost), a, s) == hipSuccess
               ? MPPI_OK
               : MPPI_EDEVICE;
}

// merge = false: rollouts only (costs, noise); merge = true: the full update,
// per MPPI iteration one fused launch (per-lane shapes) or the eight-lane
// launch and its merge launch.  Iteration i of n reads the previous
// iteration's U_new (io->U_nominal for the first), writes it to one of the
// two intermediate buffers (io->U_new and io->U_shift for the last) and
// draws with the Philox tick word n * tick + i; the global noise, when
// asked for, is the last iteration's.
int update_enqueue(mppi_solver* h, const mppi_device_io* io, hipStream_t s, void* noise, void* costs, bool merge,
                   bool want_noise)
{
    const int n = iterations_of(h->cost);
    if (n > 1 && !merge) return MPPI_ENOTSUP;
    const size_t TJ = (size_t)h->cost.T * MPPI_NJ;
    for (int i = 0; i < n; ++i) {
        mppi_device_io it = *io;
        const bool last = i == n - 1;
        it.U_nominal = i == 0 ? io->U_nominal : h->d_iter + ((i - 1) & 1) * TJ;
        if (!last) {
            it.U_new = h->d_iter + (i & 1) * TJ;
            it.U_shift = nullptr;
        }
        it.tick = io->tick * (uint64_t)n + (uint64_t)i;
        const int st = update_enqueue_one(h, &it, s, noise, costs, merge, want_noise && last);
        if (st) return st;
    }
    return MPPI_OK;
}

int weights_enqueue(mppi_solver* h, const mppi_device_io* io, hipStream_t s, const void* noise,
                    const void* costs)
{
    WeightsArgs w;
    w.costs = costs;
    w.noise = noise;
    w.U_nom = io->U_nominal;
    w.U_new = io->U_new;
    w.U_shift = io->U_shift;
    w.status = io->status;
    w.K = h->cost.K;
    w.T = h->cost.T;
    w.lambda = h->cost.lambda;
    return launch_weights(h->cost.precision, acc64_of(h->cost), w, s) == hipSuccess ? MPPI_OK : MPPI_EDEVICE;
}

int check_io(const mppi_solver* h, const mppi_device_io* io, bool need_out)
{
    if (!h || !io || !io->q || !io->qd || !io->target || !io->U_nominal) return MPPI_EINVAL;
    if (need_out && !io->U_new) return MPPI_EINVAL;
    return MPPI_OK;
}

// ---------------------------------------------------------------------------
// autotune cache: a JSON object in a file, one entry per line,
//   "<key>": {"waves_per_group": w, "groups": g, "ms": t},
// keyed by the device architecture, the problem sizes, the precision and
// the cost terms; read and rewritten whole (write to a temporary, rename)
// ---------------------------------------------------------------------------
struct TuneEntry {
    int wpg = 0, groups = 0;
    double ms = 0;
};
std::mutex g_tune_mu;
std::string g_tune_path;   // empty: no cache

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// cost terms of a problem as bits: force, orientation, wall, constant
// wrench, collision, correlated noise
unsigned cost_mask(const mppi_cost_params& c)
{
    unsigned m = has_force(c) ? 1u : 0u;
    if (c.W_ori[0] != 0.0 || c.W_ori[1] != 0.0 || c.W_ori[2] != 0.0) m |= 2u;
    if (c.ext_mode == MPPI_EXT_WALL) m |= 4u;
    if (c.ext_mode == MPPI_EXT_CONST) m |= 8u;
    if (c.n_pairs > 0) m |= 16u;
    if (c.noise_rho > 0.0) m |= 32u;
    return m;
}

std::map<std::string, TuneEntry> tune_read(const std::string& path)
{
    std::map<std::string, TuneEntry> out;
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return out;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        const char* a = std::strchr(line, '"');
        const char* b = a ? std::strchr(a + 1, '"') : nullptr;
        if (!a || !b) continue;
        TuneEntry e;
        if (std::sscanf(b + 1, " : {\"waves_per_group\": %d, \"groups\": %d, \"ms\": %lf", &e.wpg, &e.groups,
                        &e.ms) == 3)
            out[std::string(a + 1, b)] = e;
    }
    std::fclose(f);
    return out;
}

bool tune_lookup(const std::string& key, TuneEntry* e)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune_path.empty()) return false;
    const auto m = tune_read(g_tune_path);
    const auto it = m.find(key);
    if (it == m.end()) return false;
    *e = it->second;
    return true;
}

void tune_store(const std::string& key, const TuneEntry& e)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune_path.empty()) return;
    auto m = tune_read(g_tune_path);
    m[key] = e;
    const std::string tmp = g_tune_path + ".tmp" + std::to_string((long)getpid());
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : m)
        std::fprintf(f, "\"%s\": {\"waves_per_group\": %d, \"groups\": %d, \"ms\": %.6f}%s\n", kv.first.c_str(),
                     kv.second.wpg, kv.second.groups, kv.second.ms, ++i < m.size() ? "," : "");
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), g_tune_path.c_str());
    else std::remove(tmp.c_str());
}

}  // namespace

// ---------------------------------------------------------------------------
// mppi_update_noalloc: the update of mppi_update_async for callers that
// cannot allocate device memory.  Everything the update needs beyond the
// caller's inputs and outputs (the prepared model and cost, the fused
// launches' counter, the Eq. 4 partials, the intermediate sequences of
// several iterations, the costs when the caller passes none) lives in this
// file-scope array: one copy per GPU, held until the process ends, and
// shared by every call on that GPU (calls that overlap on one GPU race).
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// layout of the scratch array (byte offsets, each region 256-aligned)
constexpr size_t kSxModelF = 0, kSxModelD = 1024, kSxCostF = 3072, kSxCostD = 4096, kSxCounter = 5376,
                 kSxIter = 5632, kSxVar = kSxIter + 2 * 256 * 7 * sizeof(double);
static_assert(sizeof(ModelM<float>) <= kSxModelD - kSxModelF, "scratch layout");
static_assert(sizeof(ModelM<double>) <= kSxCostF - kSxModelD, "scratch layout");
static_assert(sizeof(CostM<float>) <= kSxCostD - kSxCostF, "scratch layout");
static_assert(sizeof(CostM<double>) <= kSxCounter - kSxCostD, "scratch layout");
static_assert(kSxVar % 256 == 0, "scratch layout");
// the prepared structs travel as kernel arguments (captured by value)
static_assert(sizeof(mppi_robot_params) + sizeof(CostM<float>) + sizeof(CostM<double>) + sizeof(void*) <= 4000,
              "kernel argument space");

// The model prepared on the device (as mppi_create does), the cost structs
// prepared on the host copied in, the fused launches' counter cleared.
__global__ void noalloc_setup_kernel(mppi_robot_params P, CostM<float> cf, CostM<double> cd,
                                     unsigned char* __restrict__ base)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        prep_model(P, *reinterpret_cast<ModelM<float>*>(base + kSxModelF));
        prep_model(P, *reinterpret_cast<ModelM<double>*>(base + kSxModelD));
        *reinterpret_cast<CostM<float>*>(base + kSxCostF) = cf;
        *reinterpret_cast<CostM<double>*>(base + kSxCostD) = cd;
        *reinterpret_cast<unsigned int*>(base + kSxCounter) = 0u;
    }
}

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kScratchDevices] = {};

size_t round256(size_t n) { return (n + 255) & ~size_t(255); }

// the scratch array's device address on the current device, looked up
// once per device (each GPU holds its own copy at its own address)
int scratch_base(unsigned char** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return MPPI_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MPPI_EDEVICE;
        g_scratch[dev] = static_cast<unsigned char*>(ptr);
    }
    *out = g_scratch[dev];
    return MPPI_OK;
}

}  // namespace

extern "C" {

int mppi_create(const mppi_robot_params* robot, const mppi_cost_params* cost, mppi_handle_t* out)
{
    if (!out) return MPPI_EINVAL;
    *out = nullptr;
    int st = validate_robot(robot);
    if (st) return st;
    st = validate_cost(cost);
    if (st) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MPPI_EDEVICE;
    mppi_solver* h = new (std::nothrow) mppi_solver;
    if (!h) return MPPI_ENOMEM;
    h->robot = *robot;
    h->cost = *cost;
    if (hipGetDevice(&h->device) != hipSuccess) { release(h); return MPPI_EDEVICE; }
    const size_t K = cost->K, T = cost->T, rs = rsize(*cost);
    const size_t io_n = kIoU + 2 * T * MPPI_NJ;
    bool ok = hipMalloc(&h->d_raw, sizeof(mppi_robot_params)) == hipSuccess &&
              hipMalloc(&h->d_mf, sizeof(ModelM<float>)) == hipSuccess &&
              hipMalloc(&h->d_md, sizeof(ModelM<double>)) == hipSuccess &&
              hipMalloc(&h->d_cf, sizeof(CostM<float>)) == hipSuccess &&
              hipMalloc(&h->d_cd, sizeof(CostM<double>)) == hipSuccess &&
              hipMalloc(&h->d_noise, K * T * MPPI_NJ * rs) == hipSuccess &&
              hipMalloc(&h->d_costs, K * rs) == hipSuccess &&
              hipMalloc(&h->d_parts, update_parts_bytes((int)K, (int)T)) == hipSuccess &&
              hipMalloc(&h->d_counter, sizeof(unsigned int)) == hipSuccess &&
              hipMalloc(&h->d_status, sizeof(int)) == hipSuccess &&
              hipMalloc(&h->d_iter, 2 * T * MPPI_NJ * sizeof(double)) == hipSuccess &&
              hipMalloc(&h->d_io, io_n * sizeof(double)) == hipSuccess &&
              hipHostMalloc(&h->h_io, io_n * sizeof(double), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&h->h_costs, K * rs, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&h->h_status, sizeof(int), hipHostMallocDefault) == hipSuccess;
    if (!ok) { release(h); return MPPI_ENOMEM; }
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) { release(h); return MPPI_EDEVICE; }
    if (hipMemset(h->d_counter, 0, sizeof(unsigned int)) != hipSuccess ||
        hipMemcpy(h->d_raw, robot, sizeof *robot, hipMemcpyHostToDevice) != hipSuccess ||
        launch_prep_model(h->d_raw, h->d_mf, h->d_md, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess || upload_cost(h) != MPPI_OK) {
        release(h);
        return MPPI_EDEVICE;
    }
    *out = h;
    return MPPI_OK;
}

int mppi_destroy(mppi_handle_t h)
{
    if (h) {
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        release(h);
    }
    return MPPI_OK;
}

int mppi_set_cost(mppi_handle_t h, const mppi_cost_params* cost)
{
    if (!h) return MPPI_EINVAL;
    int st = validate_cost(cost);
    if (st) return st;
    if (cost->K != h->cost.K || cost->T != h->cost.T || cost->precision != h->cost.precision) return MPPI_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return MPPI_EDEVICE;
    h->cost = *cost;
    return upload_cost(h);
}

int mppi_set_launch(mppi_handle_t h, int waves_per_group)
{
    if (!h || (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 8)) return MPPI_EINVAL;
    h->waves_per_group = waves_per_group;
    return MPPI_OK;
}

int mppi_set_autotune_cache(const char* path)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_path = path ? path : "";
    return MPPI_OK;
}

int mppi_autotune(mppi_handle_t h, const mppi_device_io* io, int budget_ms, void* stream, int* best_launch,
                  float* times_ms)
{
    int st = check_io(h, io, true);
    if (st) return st;
    if (budget_ms < 1) return MPPI_EINVAL;
    const int shapes[3] = {8, 2, 1};
    char key[256];
    std::snprintf(key, sizeof key, "solver|%s|K%d|T%d|%s|dyn%d|mask%02x|it%d", arch_name().c_str(), h->cost.K,
                  h->cost.T, h->cost.precision == MPPI_FP64 ? "fp64" : "fp32", h->cost.dynamics, cost_mask(h->cost),
                  iterations_of(h->cost));
    TuneEntry e;
    if (tune_lookup(key, &e) && (e.wpg == 1 || e.wpg == 2 || e.wpg == 8)) {
        h->waves_per_group = e.wpg;
        if (best_launch) *best_launch = e.wpg;
        if (times_ms)
            for (int i = 0; i < 3; ++i) times_ms[i] = -1.0f;
        return MPPI_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MPPI_EDEVICE;
    void* noise = io->noise ? io->noise : h->d_noise;
    void* costs = io->costs ? io->costs : h->d_costs;
    const int keep = h->waves_per_group;
    float best = 1e30f;
    int bw = keep;
    for (int i = 0; i < 3 && !st; ++i) {
        h->waves_per_group = shapes[i];
        // one untimed update, one timed to size the repetitions, then the
        // shape's share of the budget
        float ms = 0;
        if (update_enqueue(h, io, s, noise, costs, true, io->noise != nullptr) ||
            hipEventRecord(e0, s) != hipSuccess || update_enqueue(h, io, s, noise, costs, true, io->noise != nullptr) ||
            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = MPPI_EDEVICE; break; }
        const int reps = std::max(1, std::min(1000, (int)(budget_ms / 3.0f / std::max(ms, 1e-3f))));
        if (hipEventRecord(e0, s) != hipSuccess) { st = MPPI_EDEVICE; break; }
        for (int r = 0; r < reps && !st; ++r)
            if (update_enqueue(h, io, s, noise, costs, true, io->noise != nullptr)) st = MPPI_EDEVICE;
        if (st || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = MPPI_EDEVICE; break; }
        ms /= reps;
        if (times_ms) times_ms[i] = ms;
        if (ms < best) { best = ms; bw = shapes[i]; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->waves_per_group = st ? keep : bw;
    if (st) return st;
    if (best_launch) *best_launch = bw;
    e.wpg = bw;
    e.groups = 0;
    e.ms = best;
    tune_store(key, e);
    return MPPI_OK;
}

int mppi_rollout_async(mppi_handle_t h, const mppi_device_io* io, void* stream)
{
    int st = check_io(h, io, false);
    if (st) return st;
    return update_enqueue(h, io, (hipStream_t)stream, io->noise ? io->noise : h->d_noise,
                          io->costs ? io->costs : h->d_costs, false, true);
}

int mppi_weights_async(mppi_handle_t h, const mppi_device_io* io, void* stream)
{
    int st = check_io(h, io, true);
    if (st) return st;
    if (iterations_of(h->cost) > 1) return MPPI_ENOTSUP;
    return weights_enqueue(h, io, (hipStream_t)stream, io->noise ? io->noise : h->d_noise,
                           io->costs ? io->costs : h->d_costs);
}

int mppi_update_async(mppi_handle_t h, const mppi_device_io* io, void* stream)
{
    int st = check_io(h, io, true);
    if (st) return st;
    return update_enqueue(h, io, (hipStream_t)stream, io->noise ? io->noise : h->d_noise,
                          io->costs ? io->costs : h->d_costs, true, io->noise != nullptr);
}

int mppi_update_noalloc(const mppi_robot_params* robot, const mppi_cost_params* cost, const mppi_device_io* io,
                        void* stream)
{
    int st = validate_robot(robot);
    if (st) return st;
    st = validate_cost(cost);
    if (st) return st;
    if (!io || !io->q || !io->qd || !io->target || !io->U_nominal || !io->U_new) return MPPI_EINVAL;
    const size_t costs_bytes = io->costs ? 0 : round256((size_t)cost->K * rsize(*cost));
    const size_t need = kSxVar + costs_bytes + round256(update_parts_bytes(cost->K, cost->T));
    if (need > kScratchBytes) return MPPI_ESCRATCH;
    unsigned char* base = nullptr;
    st = scratch_base(&base);
    if (st) return st;
    CostM<float> cf;
    CostM<double> cd;
    prep_cost(*cost, cf);
    prep_cost(*cost, cd);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3(1), dim3(64), 0, s, *robot, cf, cd, base);
    if (hipGetLastError() != hipSuccess) return MPPI_EDEVICE;
    // a solver view whose buffers are regions of the scratch array (no
    // allocation; the default launch shape)
    mppi_solver h;
    h.robot = *robot;
    h.cost = *cost;
    h.d_mf = reinterpret_cast<ModelM<float>*>(base + kSxModelF);
    h.d_md = reinterpret_cast<ModelM<double>*>(base + kSxModelD);
    h.d_cf = reinterpret_cast<CostM<float>*>(base + kSxCostF);
    h.d_cd = reinterpret_cast<CostM<double>*>(base + kSxCostD);
    h.d_counter = reinterpret_cast<unsigned int*>(base + kSxCounter);
    h.d_iter = reinterpret_cast<double*>(base + kSxIter);
    h.d_costs = io->costs ? io->costs : (void*)(base + kSxVar);
    h.d_parts = base + kSxVar + costs_bytes;
    return update_enqueue(&h, io, s, io->noise, h.d_costs, true, io->noise != nullptr);
}

int mppi_update(mppi_handle_t h, const double* q, const double* qd, const mppi_target* target,
                const double* U_nominal, uint64_t seed, uint64_t tick, double* U_new, double* costs)
{
    if (!h || !q || !qd || !target || !U_nominal || !U_new) return MPPI_EINVAL;
    const int T = h->cost.T, K = h->cost.K;
    if (!finite_all(q, 7) || !finite_all(qd, 7) || !finite_all(target->p_des, 3) ||
        !finite_all(target->quat_des, 4) || !finite_all(target->F_des, 6) || !finite_all(U_nominal, T * 7))
        return MPPI_EINVAL;
    const double qn = target->quat_des[0] * target->quat_des[0] + target->quat_des[1] * target->quat_des[1] +
                      target->quat_des[2] * target->quat_des[2] + target->quat_des[3] * target->quat_des[3];
    if (!(qn > 0)) return MPPI_EINVAL;
    double* hio = h->h_io;
    std::memcpy(hio + kIoQ, q, 7 * sizeof(double));
    std::memcpy(hio + kIoQd, qd, 7 * sizeof(double));
    std::memcpy(hio + kIoTarget, target->p_des, 3 * sizeof(double));
    std::memcpy(hio + kIoTarget + 3, target->quat_des, 4 * sizeof(double));
    std::memcpy(hio + kIoTarget + 7, target->F_des, 6 * sizeof(double));
    std::memcpy(hio + kIoU, U_nominal, (size_t)T * 7 * sizeof(double));
    const size_t in_n = kIoU + (size_t)T * 7;
    hipStream_t s = h->stream;
    if (hipMemcpyAsync(h->d_io, hio, in_n * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return MPPI_EDEVICE;
    mppi_device_io io;
    std::memset(&io, 0, sizeof io);
    io.q = h->d_io + kIoQ;
    io.qd = h->d_io + kIoQd;
    io.target = h->d_io + kIoTarget;
    io.U_nominal = h->d_io + kIoU;
    io.U_new = h->d_io + in_n;
    io.status = h->d_status;
    io.seed = seed;
    io.tick = tick;
    int st = update_enqueue(h, &io, s, h->d_noise, h->d_costs, true, false);
    if (st) return st;
    if (hipMemcpyAsync(hio + in_n, h->d_io + in_n, (size_t)T * 7 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h->h_status, h->d_status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
        return MPPI_EDEVICE;
    if (costs && hipMemcpyAsync(h->h_costs, h->d_costs, (size_t)K * rsize(h->cost), hipMemcpyDeviceToHost, s) != hipSuccess)
        return MPPI_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return MPPI_EDEVICE;
    std::memcpy(U_new, hio + in_n, (size_t)T * 7 * sizeof(double));
    if (costs) {
        if (h->cost.precision == MPPI_FP64) std::memcpy(costs, h->h_costs, (size_t)K * sizeof(double));
        else
            for (int k = 0; k < K; ++k) costs[k] = (double)((const float*)h->h_costs)[k];
    }
    return *h->h_status;
}

int mppi_plant_step_wrench_async(mppi_handle_t h, double* q, double* qd, const double* u, const double* wrench,
                                 double dt, int substeps, void* stream)
{
    if (!h || !q || !qd || !u || !(dt > 0) || substeps < 1) return MPPI_EINVAL;
    return launch_plant(h->d_md, h->d_cd, q, qd, u, dt, substeps, wrench, (hipStream_t)stream) == hipSuccess
               ? MPPI_OK
               : MPPI_EDEVICE;
}

int mppi_plant_step_async(mppi_handle_t h, double* q, double* qd, const double* u, double dt, int substeps,
                          void* stream)
{
    return mppi_plant_step_wrench_async(h, q, qd, u, nullptr, dt, substeps, stream);
}

int mppi_ee_pose_async(mppi_handle_t h, const double* q, int n, double* pose, void* stream)
{
    if (!h || !q || !pose || n < 1) return MPPI_EINVAL;
    return launch_ee_pose(h->d_md, q, n, pose, (hipStream_t)stream) == hipSuccess ? MPPI_OK : MPPI_EDEVICE;
}

int mppi_select_nominal_async(mppi_handle_t h, const mppi_device_io* io, const double* U_candidate, double* costs,
                              void* stream)
{
    if (check_io(h, io, false) || !U_candidate) return MPPI_EINVAL;
    const bool fp64 = h->cost.precision == MPPI_FP64;
    return launch_select(h->cost.precision, has_force(h->cost), h->cost.n_pairs > 0,
                         fp64 ? (const void*)h->d_md : (const void*)h->d_mf,
                         fp64 ? (const void*)h->d_cd : (const void*)h->d_cf, io->q, io->qd, io->target,
                         const_cast<double*>(io->U_nominal), U_candidate, h->cost.T, costs,
                         (hipStream_t)stream) == hipSuccess
               ? MPPI_OK
               : MPPI_EDEVICE;
}

int mppi_warm_start_async(mppi_handle_t h, const double* U_new, double* U_out, double shift_steps, void* stream)
{
    if (!h || !U_new || !U_out || !std::isfinite(shift_steps) || shift_steps < 0 || shift_steps > h->cost.T)
        return MPPI_EINVAL;
    if (ranges_overlap(U_new, U_out, (size_t)h->cost.T * MPPI_NJ)) return MPPI_EINVAL;
    return launch_warm_start(U_new, U_out, h->cost.T, shift_steps, (hipStream_t)stream) == hipSuccess ? MPPI_OK
                                                                                                      : MPPI_EDEVICE;
}

const char* mppi_strerror(int status)
{
    switch (status) {
    case MPPI_OK: return "ok";
    case MPPI_EINVAL: return "invalid argument";
    case MPPI_ENONFINITE: return "all sample costs non-finite";
    case MPPI_ENOMEM: return "out of memory";
    case MPPI_EDEVICE: return "device error";
    case MPPI_ENOTSUP: return "not supported";
    case MPPI_ESCRATCH: return "request exceeds the static workspace of mppi_update_noalloc";
    default: return "unknown status";
    }
}

const char* mppi_version(void) { return "mppi-gfx950 0.1"; }

}  // extern "C"

// ---------------------------------------------------------------------------
// batched problems
// ---------------------------------------------------------------------------
#include <vector>


struct mppi_batch {
    int n = 0;
    std::vector<mppi_robot_params> robot;
    std::vector<mppi_cost_params> cost;
    std::vector<size_t> u_off, k_off;
    size_t u_total = 0, k_total = 0;
    mppi_robot_params* d_raw = nullptr;
    ModelM<float>* d_mf = nullptr;
    ModelM<double>* d_md = nullptr;
    CostM<float>* d_cf = nullptr;
    CostM<double>* d_cd = nullptr;   // the FP64 plant's wall and external force
    void* d_probs = nullptr;
    int2* d_items = nullptr;
    int nitems = 0;
    unsigned int* d_sync = nullptr;   // queue, done, counters[n]
    double* d_parts = nullptr;
    uint64_t* d_tick = nullptr;   // [0]: graph replays (advanced by the graph), [1]: eager launches
    int wpg = 1, groups = 1024;
    int collision = 0;            // some problem has the collision term
    int iterations = 1;           // MPPI iterations per update (the same for every problem)
    double* d_iter = nullptr;     // [2][u_total]: U of the intermediate iterations
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
};

namespace {

void batch_release(mppi_batch* b)
{
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    (void)hipFree(b->d_raw);
    (void)hipFree(b->d_mf);
    (void)hipFree(b->d_md);
    (void)hipFree(b->d_cf);
    (void)hipFree(b->d_cd);
    (void)hipFree(b->d_probs);
    (void)hipFree(b->d_items);
    (void)hipFree(b->d_sync);
    (void)hipFree(b->d_parts);
    (void)hipFree(b->d_iter);
    (void)hipFree(b->d_tick);
    delete b;
}

BatchArgs batch_args(mppi_batch* b, const mppi_batch_io* io, const uint64_t* tick_slot)
{
    BatchArgs a;
    a.probs = b->d_probs;
    a.models = b->d_mf;
    a.items = b->d_items;
    a.nitems = b->nitems;
    a.queue = b->d_sync;
    a.done = b->d_sync + 1;
    a.counters = b->d_sync + 2;
    a.q = io->q;
    a.qd = io->qd;
    a.target = io->target;
    a.U_nom = io->U_nominal;
    a.U_new = io->U_new;
    a.U_shift = io->U_shift;
    a.costs = io->costs;
    a.status = io->status;
    a.seeds = io->seed;
    a.tick = tick_slot;
    a.parts = b->d_parts;
    a.collision = b->collision;
    a.iter = 0;
    a.niter = 1;
    return a;
}

// The update as b->iterations chained launches: iteration i reads the
// previous one's U_new (io->U_nominal for the first), writes one of two
// intermediate buffers (io->U_new and io->U_shift for the last) and draws
// with the Philox tick word iterations * tick + i (tick read from tick_slot
// on the device, so a captured graph replays it).
bool enqueue_batch_iterations(mppi_batch* b, const mppi_batch_io* io, const uint64_t* tick_slot, hipStream_t s)
{
    const int n = b->iterations;
    for (int i = 0; i < n; ++i) {
        BatchArgs a = batch_args(b, io, tick_slot);
        a.iter = i;
        a.niter = n;
        if (i > 0) a.U_nom = b->d_iter + (size_t)((i - 1) & 1) * b->u_total;
        if (i < n - 1) {
            a.U_new = b->d_iter + (size_t)(i & 1) * b->u_total;
            a.U_shift = nullptr;
        }
        if (launch_batch(a, b->wpg, b->groups, s) != hipSuccess) return false;
    }
    return true;
}

int check_batch_io(const mppi_batch* b, const mppi_batch_io* io)
{
    if (!b || !io || !io->q || !io->qd || !io->target || !io->U_nominal || !io->U_new || !io->seed)
        return MPPI_EINVAL;
    return MPPI_OK;
}

}  // namespace

extern "C" {

int mppi_batch_create(const mppi_problem_desc* descs, int n, mppi_batch_t* out)
{
    if (!out) return MPPI_EINVAL;
    *out = nullptr;
    if (!descs || n < 1 || n > (1 << 16)) return MPPI_EINVAL;
    for (int p = 0; p < n; ++p) {
        int st = validate_robot(descs[p].robot);
        if (!st) st = validate_cost(descs[p].cost);
        if (st) return st;
        if (descs[p].cost->precision != MPPI_FP32 || descs[p].cost->T > kMaxTBatch ||
            descs[p].cost->dynamics != MPPI_DYN_ABA ||
            iterations_of(*descs[p].cost) != iterations_of(*descs[0].cost))
            return MPPI_ENOTSUP;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MPPI_EDEVICE;
    mppi_batch* b = new (std::nothrow) mppi_batch;
    if (!b) return MPPI_ENOMEM;
    b->n = n;
    b->iterations = iterations_of(*descs[0].cost);
    b->robot.resize(n);
    b->cost.resize(n);
    b->u_off.resize(n);
    b->k_off.resize(n);
    std::vector<long long> part_off(n);
    std::vector<int> ntiles(n);
    long long parts_total = 0;
    for (int p = 0; p < n; ++p) {
        b->robot[p] = *descs[p].robot;
        b->cost[p] = *descs[p].cost;
        if (b->cost[p].n_pairs > 0) b->collision = 1;
        const int K = b->cost[p].K, T = b->cost[p].T;
        b->u_off[p] = b->u_total;
        b->k_off[p] = b->k_total;
        b->u_total += (size_t)T * MPPI_NJ;
        b->k_total += (size_t)K;
        ntiles[p] = (K + 63) / 64;
        part_off[p] = parts_total;
        parts_total += (long long)ntiles[p] * (2 + T * MPPI_NJ);
    }
    // work list: 64-sample tiles, heaviest per-tile work (horizon, force
    // cost) first, so the long rollouts start early (longest-processing-time
    // order)
    std::vector<int> order(n);
    for (int p = 0; p < n; ++p) order[p] = p;
    auto work = [&](int p) { return (double)b->cost[p].T * (has_force(b->cost[p]) ? 1.25 : 1.0); };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
    std::vector<int2> items;
    for (int p : order)
        for (int t = 0; t < ntiles[p]; ++t) items.push_back(make_int2(p, t));
    b->nitems = (int)items.size();
    bool ok = hipMalloc(&b->d_raw, sizeof(mppi_robot_params) * n) == hipSuccess &&
              hipMalloc(&b->d_mf, sizeof(ModelM<float>) * n) == hipSuccess &&
              hipMalloc(&b->d_md, sizeof(ModelM<double>) * n) == hipSuccess &&
              hipMalloc(&b->d_cf, sizeof(CostM<float>) * n) == hipSuccess &&
              hipMalloc(&b->d_cd, sizeof(CostM<double>) * n) == hipSuccess &&
              hipMalloc(&b->d_probs, batch_problem_bytes() * n) == hipSuccess &&
              hipMalloc(&b->d_items, sizeof(int2) * items.size()) == hipSuccess &&
              hipMalloc(&b->d_sync, sizeof(unsigned int) * (2 + n)) == hipSuccess &&
              hipMalloc(&b->d_parts, sizeof(double) * parts_total) == hipSuccess &&
              hipMalloc(&b->d_iter, sizeof(double) * 2 * b->u_total) == hipSuccess &&
              hipMalloc(&b->d_tick, 2 * sizeof(uint64_t)) == hipSuccess;
    if (!ok) { batch_release(b); return MPPI_ENOMEM; }
    std::vector<CostM<float>> cf(n);
    std::vector<CostM<double>> cd(n);
    std::vector<char> probs(batch_problem_bytes() * n);
    for (int p = 0; p < n; ++p) {
        prep_cost(b->cost[p], cf[p]);
        prep_cost(b->cost[p], cd[p]);
        const mppi_cost_params& c = b->cost[p];
        fill_batch_problem(probs.data() + batch_problem_bytes() * p, b->d_mf + p, b->d_cf + p, b->d_md + p,
                           b->d_cd + p, c.K, c.T, has_force(c) ? 1 : 0, acc64_of(c) ? 1 : 0, c.n_pairs > 0 ? 1 : 0,
                           c.lambda, ntiles[p],
                           (long long)b->u_off[p], (long long)b->k_off[p], part_off[p]);
    }
    ok = hipMemcpy(b->d_raw, b->robot.data(), sizeof(mppi_robot_params) * n, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_cf, cf.data(), sizeof(CostM<float>) * n, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_cd, cd.data(), sizeof(CostM<double>) * n, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_probs, probs.data(), probs.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(b->d_sync, 0, sizeof(unsigned int) * (2 + n)) == hipSuccess &&
         hipMemset(b->d_tick, 0, 2 * sizeof(uint64_t)) == hipSuccess;
    for (int p = 0; ok && p < n; ++p)
        ok = launch_prep_model(b->d_raw + p, b->d_mf + p, b->d_md + p, nullptr) == hipSuccess;
    if (!ok || hipDeviceSynchronize() != hipSuccess) { batch_release(b); return MPPI_EDEVICE; }
    *out = b;
    return MPPI_OK;
}

int mppi_batch_destroy(mppi_batch_t b)
{
    if (b) {
        (void)hipDeviceSynchronize();
        batch_release(b);
    }
    return MPPI_OK;
}

int mppi_batch_layout(mppi_batch_t b, size_t* u_off, size_t* k_off, size_t* u_total, size_t* k_total)
{
    if (!b) return MPPI_EINVAL;
    for (int p = 0; p < b->n; ++p) {
        if (u_off) u_off[p] = b->u_off[p];
        if (k_off) k_off[p] = b->k_off[p];
    }
    if (u_total) *u_total = b->u_total;
    if (k_total) *k_total = b->k_total;
    return MPPI_OK;
}

int mppi_batch_plant_step_async(mppi_batch_t b, const mppi_batch_io* io, double dt, int substeps, void* stream)
{
    if (check_batch_io(b, io) || !(dt > 0) || substeps < 1) return MPPI_EINVAL;
    return launch_batch_plant(b->d_probs, b->n, const_cast<double*>(io->q), const_cast<double*>(io->qd), io->U_new,
                              dt, substeps, (hipStream_t)stream) == hipSuccess
               ? MPPI_OK
               : MPPI_EDEVICE;
}

int mppi_batch_select_nominal_async(mppi_batch_t b, const mppi_batch_io* io, const double* U_candidates,
                                    double* costs, void* stream)
{
    if (check_batch_io(b, io) || !U_candidates) return MPPI_EINVAL;
    return launch_batch_select(b->d_probs, b->n, io->q, io->qd, io->target, const_cast<double*>(io->U_nominal),
                               U_candidates, costs, (hipStream_t)stream) == hipSuccess
               ? MPPI_OK
               : MPPI_EDEVICE;
}

int mppi_batch_warm_start_async(mppi_batch_t b, const double* U_new, double* U_out, double shift_steps,
                                void* stream)
{
    if (!b || !U_new || !U_out || !std::isfinite(shift_steps) || shift_steps < 0 || shift_steps > kMaxTBatch)
        return MPPI_EINVAL;
    if (ranges_overlap(U_new, U_out, b->u_total)) return MPPI_EINVAL;
    return launch_batch_warm_start(b->d_probs, b->n, U_new, U_out, shift_steps, (hipStream_t)stream) == hipSuccess
               ? MPPI_OK
               : MPPI_EDEVICE;
}

int mppi_batch_set_launch(mppi_batch_t b, int waves_per_group, int groups)
{
    if (!b || (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4 && waves_per_group != 8) ||
        groups < 1 || groups > (1 << 16))
        return MPPI_EINVAL;
    b->wpg = waves_per_group;
    b->groups = groups;
    return MPPI_OK;
}

int mppi_batch_set_tick(mppi_batch_t b, uint64_t tick)
{
    if (!b) return MPPI_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return MPPI_EDEVICE;
    return hipMemcpy(b->d_tick, &tick, sizeof tick, hipMemcpyHostToDevice) == hipSuccess ? MPPI_OK : MPPI_EDEVICE;
}

int mppi_batch_update_async(mppi_batch_t b, const mppi_batch_io* io, uint64_t tick, void* stream)
{
    int st = check_batch_io(b, io);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (launch_set_tick(b->d_tick + 1, tick, s) != hipSuccess) return MPPI_EDEVICE;
    return enqueue_batch_iterations(b, io, b->d_tick + 1, s) ? MPPI_OK : MPPI_EDEVICE;
}

int mppi_batch_autotune(mppi_batch_t b, const mppi_batch_io* io, int reps, void* stream, int* best_wpg,
                        int* best_groups, float* times_ms)
{
    int st = check_batch_io(b, io);
    if (st) return st;
    if (reps < 1) return MPPI_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    constexpr int kShapes = 16;
    const int wpgs[4] = {1, 2, 4, 8};
    const int waves[4] = {256, 512, 1024, 2048};
    // cache key: architecture, total sample-steps (power-of-two bucket),
    // horizon range, precision, union of the problems' cost terms, iterations
    long long kt = 0;
    int tmin = 1 << 30, tmax = 0;
    unsigned mask = 0;
    for (int p = 0; p < b->n; ++p) {
        kt += (long long)b->cost[p].K * b->cost[p].T;
        tmin = std::min(tmin, b->cost[p].T);
        tmax = std::max(tmax, b->cost[p].T);
        mask |= cost_mask(b->cost[p]);
    }
    int lg = 0;
    while ((2LL << lg) <= kt) ++lg;
    char key[256];
    std::snprintf(key, sizeof key, "batch|%s|kt2^%d|T%d-%d|fp32|mask%02x|it%d", arch_name().c_str(), lg, tmin, tmax,
                  mask, b->iterations);
    TuneEntry e;
    if (tune_lookup(key, &e) && (e.wpg == 1 || e.wpg == 2 || e.wpg == 4 || e.wpg == 8) && e.groups >= 1 &&
        e.groups <= (1 << 16)) {
        b->wpg = e.wpg;
        b->groups = e.groups;
        if (best_wpg) *best_wpg = e.wpg;
        if (best_groups) *best_groups = e.groups;
        if (times_ms)
            for (int i = 0; i < kShapes; ++i) times_ms[i] = -1.0f;
        return MPPI_OK;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MPPI_EDEVICE;
    BatchArgs a = batch_args(b, io, b->d_tick + 1);
    float best = 1e30f;
    int bw = b->wpg, bg = b->groups, idx = 0;
    st = MPPI_OK;
    for (int wi = 0; wi < 4 && !st; ++wi)
        for (int vi = 0; vi < 4 && !st; ++vi, ++idx) {
            const int w = wpgs[wi], g = waves[vi] / w;
            // one untimed launch, then `reps` timed ones
            if (launch_set_tick(b->d_tick + 1, 0, s) != hipSuccess || launch_batch(a, w, g, s) != hipSuccess ||
                hipEventRecord(e0, s) != hipSuccess) { st = MPPI_EDEVICE; break; }
            for (int r = 0; r < reps; ++r)
                if (launch_set_tick(b->d_tick + 1, (uint64_t)r + 1, s) != hipSuccess ||
                    launch_batch(a, w, g, s) != hipSuccess) { st = MPPI_EDEVICE; break; }
            float ms = 0;
            if (st || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = MPPI_EDEVICE; break; }
            ms /= reps;
            if (times_ms) times_ms[idx] = ms;
            if (ms < best) { best = ms; bw = w; bg = g; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    b->wpg = bw;
    b->groups = bg;
    if (best_wpg) *best_wpg = bw;
    if (best_groups) *best_groups = bg;
    e.wpg = bw;
    e.groups = bg;
    e.ms = best;
    tune_store(key, e);
    return MPPI_OK;
}

int mppi_batch_graph_capture(mppi_batch_t b, const mppi_batch_io* io)
{
    int st = check_batch_io(b, io);
    if (st) return st;
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return MPPI_EDEVICE;
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    ok = ok && enqueue_batch_iterations(b, io, b->d_tick, cs);
    ok = ok && launch_advance_tick(b->d_tick, cs) == hipSuccess;
    hipGraph_t g = nullptr;
    ok = (hipStreamEndCapture(cs, &g) == hipSuccess) && ok && g;
    (void)hipStreamDestroy(cs);
    if (!ok) { if (g) (void)hipGraphDestroy(g); return MPPI_EDEVICE; }
    b->graph = g;
    if (hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        b->graph = nullptr;
        b->gexec = nullptr;
        return MPPI_EDEVICE;
    }
    return MPPI_OK;
}

int mppi_batch_graph_launch(mppi_batch_t b, void* stream)
{
    if (!b || !b->gexec) return MPPI_EINVAL;
    return hipGraphLaunch(b->gexec, (hipStream_t)stream) == hipSuccess ? MPPI_OK : MPPI_EDEVICE;
}

}  // extern "C"
