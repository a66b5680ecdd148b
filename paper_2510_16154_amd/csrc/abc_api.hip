// Host side of the C ABI declared in include/abc.h: argument checks, workspace
// carving, the forward and adjoint sweeps, and the solver loop (method of
// multipliers, Alg. 2, with the direct-adjoint / two-way Armijo control argmin
// of Alg. 1).  Decisions of the line search are taken in FP64 on the host from
// FP32 device reductions.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/abc.h"
#include "abc_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define ABC_HIP(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(ABC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

// A named range on the profiler's marker trace (rocprofv3 --marker-trace) for the
// lifetime of the object; without a profiler the calls return at once.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Sequential bump allocator over the caller's workspace.
struct Carve {
    char* base;
    size_t used = 0;
    explicit Carve(void* b) : base((char*)b) {}
    template <class T>
    T* take(size_t count) {
        T* p = base ? (T*)(base + used) : nullptr;
        used += align_up(count * sizeof(T));
        return p;
    }
};

// Pinned host array owned for the duration of a call; copies from it are
// queued on `st`, which is drained before the array is freed.
template <class T>
struct PinnedHost {
    T* ptr = nullptr;
    hipStream_t st = nullptr;
    PinnedHost() = default;
    PinnedHost(const PinnedHost&) = delete;
    PinnedHost& operator=(const PinnedHost&) = delete;
    ~PinnedHost() {
        if (!ptr) return;
        (void)hipStreamSynchronize(st);
        (void)hipHostFree(ptr);
    }
    int alloc(size_t n) {
        ABC_HIP(hipHostMalloc((void**)&ptr, std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault));
        return ABC_OK;
    }
};

// Captured HIP graphs of sweep launches, keyed by the caller.  A sweep is
// recorded once on a private capture stream and replayed on the caller's
// stream; kernels read controls, job tables and buffers through pointers
// that stay fixed, so one recording serves every replay.  The key must name
// everything a recorded launch depends on (buffers, sizes, launch shapes and
// scalar arguments).  A cache with max_entries > 0 drops all its graphs
// (after draining the stream) before it would hold more.
struct GraphCache {
    hipStream_t cap = nullptr;
    hipStream_t last = nullptr;
    size_t max_entries = 0;
    std::map<std::vector<long>, hipGraphExec_t> execs;
    GraphCache() = default;
    GraphCache(const GraphCache&) = delete;
    GraphCache& operator=(const GraphCache&) = delete;
    ~GraphCache() {
        if (last) (void)hipStreamSynchronize(last);
        for (auto& kv : execs) (void)hipGraphExecDestroy(kv.second);
        if (cap) (void)hipStreamDestroy(cap);
    }
    template <class F>
    int run(bool enabled, const std::vector<long>& key, hipStream_t st, F&& record) {
        last = st;
        if (!enabled) return record(st);
        auto it = execs.find(key);
        if (it == execs.end() && max_entries > 0 && execs.size() >= max_entries) {
            ABC_HIP(hipStreamSynchronize(st));
            for (auto& kv : execs) (void)hipGraphExecDestroy(kv.second);
            execs.clear();
        }
        if (it == execs.end()) {
            if (!cap) ABC_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            ABC_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            const int rc = record(cap);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(cap, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(ABC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            hipGraphExec_t ex = nullptr;
            const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e2 != hipSuccess) return fail(ABC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
            it = execs.emplace(key, ex).first;
        }
        ABC_HIP(hipGraphLaunch(it->second, st));
        return ABC_OK;
    }
};

// Sweep graphs of abc_solve, kept per host thread across calls (a solve
// records six: three trajectory buffers forward, three adjoint).  Never
// destroyed: the process end reclaims them, and no HIP call runs at exit.
GraphCache& solve_graphs() {
    thread_local GraphCache* g = nullptr;
    if (!g) {
        g = new GraphCache;
        g->max_entries = 48;
    }
    return *g;
}

long float_bits(float x) {
    uint32_t u;
    std::memcpy(&u, &x, sizeof(u));
    return (long)u;
}

// Columns of abc_solve_log.phi_out per DAL iteration.
constexpr int kStepLog = 5;

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

struct Shape {
    int H, W, C;
    size_t npix() const { return (size_t)H * W; }
    size_t field() const { return npix() * C; }
    double area() const { return (1.0 / W) * (1.0 / H); }
};

float norm_factor(const abc_params* p, const Shape& s) {
    if (p->inv_norm > 0.0f) return p->inv_norm;
    const double win = (double)(2 * p->R + 1) * (double)(2 * p->R + 1);
    return (float)(1.0 / std::min((double)s.npix(), win));
}

int check_shape(int H, int W, int C) {
    if (H < 1 || W < 1) return fail(ABC_EINVAL, "H and W must be >= 1");
    if (C < 1 || C > ABC_MAX_CHANNELS) return fail(ABC_EINVAL, "C must be in [1, 64]");
    if ((double)H * (double)W * (double)C > 4.0e9) return fail(ABC_EINVAL, "H * W * C must be <= 4e9");
    return ABC_OK;
}

int check_params(const abc_params* p) {
    if (!p) return fail(ABC_EINVAL, "params is NULL");
    if (p->K < 1) return fail(ABC_EINVAL, "K must be >= 1");
    if ((p->R < 0 || p->R > ABC_MAX_DIRECT_RADIUS) && p->R != ABC_RADIUS_SUPPORT)
        return fail(ABC_EINVAL, "R must be in [0, 32767] or ABC_RADIUS_SUPPORT");
    if (!(p->dt > 0.0f) || !std::isfinite(p->dt)) return fail(ABC_EINVAL, "dt must be > 0");
    if (!(p->inv_norm >= 0.0f)) return fail(ABC_EINVAL, "inv_norm must be >= 0");
    for (int m = 0; m < 2; ++m) {
        if (!(p->eps_min[m] >= 0.0f) || !(p->eps_min[m] <= p->eps_max[m]) || !std::isfinite(p->eps_max[m]))
            return fail(ABC_EINVAL, "control box must satisfy 0 <= eps_min <= eps_max < inf");
    }
    if (!(p->rho > 0.0f)) return fail(ABC_EINVAL, "rho must be > 0");
    if (!(p->alpha >= 0.0f) || !(p->gamma >= 0.0f)) return fail(ABC_EINVAL, "alpha and gamma must be >= 0");
    if (p->max_outer < 0 || p->max_inner < 0 || p->max_ls < 1)
        return fail(ABC_EINVAL, "max_outer, max_inner >= 0 and max_ls >= 1 required");
    if (!(p->sigma0 > 0.0) || !(p->armijo_b > 0.0 && p->armijo_b < 1.0) ||
        !(p->armijo_c > 0.0 && p->armijo_c < 1.0))
        return fail(ABC_EINVAL, "Armijo parameters: sigma0 > 0, b and c in (0,1)");
    if (p->ckpt_every < 0) return fail(ABC_EINVAL, "ckpt_every must be >= 0");
    if (p->cost != ABC_COST_TV && p->cost != ABC_COST_QUADRATIC) return fail(ABC_EINVAL, "unknown cost");
    if (p->flags & ~(ABC_FLAG_NO_GRAPHS | ABC_FLAG_AUTOTUNE | ABC_FLAG_PERSISTENT))
        return fail(ABC_EINVAL, "unknown flag bits");
    if (!(p->stop_K >= 0.0)) return fail(ABC_EINVAL, "stop_K must be >= 0");
    if (!(p->tol_gap >= 0.0)) return fail(ABC_EINVAL, "tol_gap must be >= 0");
    return ABC_OK;
}

// p with R resolved for an H x W image when it asks for the support radius
// (ABC_RADIUS_SUPPORT), p itself otherwise.  Call after check_params.
const abc_params* with_radius(const abc_params* p, int H, int W, abc_params& tmp) {
    if (p->R != ABC_RADIUS_SUPPORT) return p;
    tmp = *p;
    int32_t r = 0;
    (void)abc_support_radius(H, W, p->eps_min[0], &r);
    tmp.R = r;
    return &tmp;
}

int pick_tile(const abc_params* p, int C, int fields, abc::Tile* t) {
    int tx = p->tile_x, ty = p->tile_y;
    if (fields == 2 && (p->adj_tile_x > 0 || p->adj_tile_y > 0)) {
        tx = p->adj_tile_x;
        ty = p->adj_tile_y;
    }
    if (tx > 0 || ty > 0) {
        abc::Tile u{tx, ty};
        if (!abc::tile_ok(C, p->R, u, fields))
            return fail(ABC_EINVAL, "tile: tile_y must be a multiple of the pixels per thread (" +
                                        std::to_string(abc::rows_per_thread(C, p->R)) +
                                        "), tile_x * tile_y / that a multiple of 64 and <= 256, and fit in LDS");
        *t = u;
        return ABC_OK;
    }
    *t = abc::default_tile(C, p->R, fields);
    if (t->tx == 0) return fail(ABC_EINVAL, "no interaction tile fits this channel count and radius");
    return ABC_OK;
}

int traj_slots(const abc_params* p) {
    if (p->ckpt_every <= 0) return p->K + 1;
    return (p->K + p->ckpt_every - 1) / p->ckpt_every + 1;
}

// ---------------------------------------------------------------------------
// Workspace layouts.

struct AdjointWs {
    float* pa;     // adjoint ping
    float* pb;     // adjoint pong
    double* part;  // K x tiles x 2 (FP64 gradient partials)
    float* seg;   // (ckpt_every + 1) fields when checkpointed
};

AdjointWs carve_adjoint(Carve& cv, const Shape& s, const abc_params* p, int tiles) {
    AdjointWs w;
    w.pa = cv.take<float>(s.field());
    w.pb = cv.take<float>(s.field());
    w.part = cv.take<double>((size_t)p->K * tiles * 2);
    w.seg = p->ckpt_every > 0 ? cv.take<float>((size_t)(p->ckpt_every + 1) * s.field()) : nullptr;
    return w;
}

struct PdWs {
    float* part;  // pd_blocks x kPdQuantities
    float* out;   // kPdQuantities
    int* flag;
};

PdWs carve_pd(Carve& cv, const Shape& s) {
    PdWs w;
    w.part = cv.take<float>((size_t)abc::pd_blocks(s.H, s.W) * abc::kPdQuantities);
    w.out = cv.take<float>(abc::kPdQuantities);
    w.flag = cv.take<int>(1);
    return w;
}

struct SolveWs {
    float* traj[3];
    float* eps[3];
    float* v;
    float* mu;
    double* G;  // K x 2 reduced control gradient sums
    AdjointWs adj;
    PdWs pd;
};

SolveWs carve_solve(Carve& cv, const Shape& s, const abc_params* p, int tiles) {
    SolveWs w;
    for (int i = 0; i < 3; ++i) w.traj[i] = cv.take<float>((size_t)(p->K + 1) * s.field());
    for (int i = 0; i < 3; ++i) w.eps[i] = cv.take<float>((size_t)p->K * 2);
    w.v = cv.take<float>(2 * s.field());
    w.mu = cv.take<float>(2 * s.field());
    w.G = cv.take<double>((size_t)p->K * 2);
    abc_params q = *p;
    q.ckpt_every = 0;
    w.adj = carve_adjoint(cv, s, &q, tiles);
    w.pd = carve_pd(cv, s);
    return w;
}

size_t ws_bytes_for(int kind, const Shape& s, const abc_params* p, const abc::Tile& tf, const abc::Tile& ta) {
    Carve cv(nullptr);
    switch (kind) {
        case ABC_WS_SOLVE: carve_solve(cv, s, p, abc::adj_part_count(s.H, s.W, s.C, p->R, ta)); break;
        case ABC_WS_FORWARD:
            if (p->ckpt_every > 0) cv.take<float>(2 * s.field());
            break;
        case ABC_WS_ADJOINT: carve_adjoint(cv, s, p, abc::adj_part_count(s.H, s.W, s.C, p->R, ta)); break;
        case ABC_WS_PD: carve_pd(cv, s); break;
        default: return 0;
    }
    (void)tf;
    return cv.used;
}

// ---------------------------------------------------------------------------
// Sweeps.

int forward_steps(const float* cin, float* const* dst, int k0, int k1, const float* eps, const Shape& s,
                  const abc_params* p, float dts, abc::Tile t, hipStream_t st) {
    // dst[k - k0] receives c^{k+1} for k in [k0, k1); cin is c^{k0}.
    const float* cur = cin;
    for (int k = k0; k < k1; ++k) {
        float* out = dst[k - k0];
        ABC_HIP(abc::launch_forward_step(cur, out, eps, k, s.H, s.W, s.C, p->R, dts, t, st));
        cur = out;
    }
    return ABC_OK;
}

// Full trajectory: traj holds K+1 fields, traj[0] = c0.
int forward_sweep_full(const float* c0, float* traj, const float* eps, const Shape& s, const abc_params* p,
                       float dts, abc::Tile t, hipStream_t st) {
    const size_t f = s.field();
    if (traj != c0) ABC_HIP(hipMemcpyAsync(traj, c0, f * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (p->R == 0) {
        for (int k = 1; k <= p->K; ++k)
            ABC_HIP(hipMemcpyAsync(traj + k * f, c0, f * sizeof(float), hipMemcpyDeviceToDevice, st));
        return ABC_OK;
    }
    for (int k = 0; k < p->K; ++k)
        ABC_HIP(abc::launch_forward_step(traj + k * f, traj + (k + 1) * f, eps, k, s.H, s.W, s.C, p->R, dts, t, st));
    return ABC_OK;
}

// Adjoint over steps [k0, k1) of a stored trajectory segment: states[k - k0] = c^k.
// pin holds p^{k1}; the result p^{k0} ends in *pout_final (one of pa / pb).
int adjoint_steps(const float* const* states, int k0, int k1, const float* eps, const Shape& s,
                  const abc_params* p, float dts, abc::Tile t, float*& cur, float*& spare, double* part,
                  int tiles, hipStream_t st) {
    for (int k = k1 - 1; k >= k0; --k) {
        ABC_HIP(abc::launch_adjoint_step(states[k - k0], cur, spare, eps, k, s.H, s.W, s.C, p->R, dts, t,
                                         part + (size_t)k * tiles * 2, st));
        std::swap(cur, spare);
    }
    return ABC_OK;
}

// Pinned host floats for the scalar reads that the solver waits on (objective,
// energies): one array per host thread, allocated on its first use and kept
// until the process ends.  A read into pinned memory returns about 7 us sooner
// than one into pageable memory.  NULL if the allocation failed (callers then
// read into their own stack array).
constexpr int kReadbackFloats = 16;
static_assert(abc::kTermQuantities <= kReadbackFloats && abc::kPdQuantities <= kReadbackFloats, "readback size");
float* scalar_readback() {
    thread_local float* buf = nullptr;
    thread_local bool tried = false;
    if (!tried) {
        tried = true;
        if (hipHostMalloc((void**)&buf, kReadbackFloats * sizeof(float), hipHostMallocDefault) != hipSuccess) {
            buf = nullptr;
            (void)hipGetLastError();
        }
    }
    return buf;
}

// Terminal condition (pK may be NULL) and, when phi is set, the objective L~ and
// the TV energy K = TV + fidelity of cK (Kout, TVout, fidout may be NULL).
int objective(const float* cK, const float* c0, const float* v, const float* mu, float* pK, const Shape& s,
              const abc_params* p, const PdWs& w, hipStream_t st, double* phi, double* Kout = nullptr,
              double* TVout = nullptr, double* fidout = nullptr) {
    ABC_HIP(abc::launch_terminal(cK, c0, v, mu, s.H, s.W, s.C, p->rho, p->alpha, (float)s.area(), pK, w.part, st));
    if (!phi) return ABC_OK;
    ABC_HIP(abc::launch_reduce_rows(w.part, 1, abc::pd_blocks(s.H, s.W), abc::kTermQuantities, w.out, 1.0f, st));
    float local[abc::kTermQuantities];
    float* h = scalar_readback();
    if (!h) h = local;
    ABC_HIP(hipMemcpyAsync(h, w.out, abc::kTermQuantities * sizeof(float), hipMemcpyDeviceToHost, st));
    ABC_HIP(hipStreamSynchronize(st));
    *phi = s.area() * (double)h[0];
    const double tv = s.area() * (double)h[1], fid = s.area() * 0.5 * (double)p->alpha * (double)h[2];
    if (Kout) *Kout = tv + fid;
    if (TVout) *TVout = tv;
    if (fidout) *fidout = fid;
    return ABC_OK;
}

void energies_from(const float* q, const Shape& s, const abc_params* p, abc_stats* out) {
    const double a = s.area();
    const double svg = q[0], sg = q[1], sv = q[2], tv = q[3], sf = q[4], lp = q[5], ltp = q[6];
    out->TV = a * tv;
    out->fid = a * 0.5 * (double)p->alpha * sf;
    out->K = out->TV + out->fid;
    out->L = a * (lp + 0.5 * (double)p->rho * svg + 0.5 * (double)p->alpha * sf);
    out->Ltilde = a * (ltp + 0.5 * (double)p->alpha * sf);
    out->r_abs = std::sqrt(a * svg);
    const double den = std::max({std::sqrt(sg), std::sqrt(sv), 1e-30});
    out->r_rel = std::sqrt(svg) / den;
}

int pd_update(const float* cK, const float* c0, float* v, float* mu, int update_mu, const Shape& s,
              const abc_params* p, const PdWs& w, hipStream_t st, abc_stats* out) {
    ABC_HIP(abc::launch_pd_step(cK, c0, v, mu, update_mu, s.H, s.W, s.C, p->rho, p->gamma, w.part, st));
    if (!out) return ABC_OK;
    ABC_HIP(abc::launch_reduce_rows(w.part, 1, abc::pd_blocks(s.H, s.W), abc::kPdQuantities, w.out, 1.0f, st));
    float local[abc::kPdQuantities];
    float* q = scalar_readback();
    if (!q) q = local;
    ABC_HIP(hipMemcpyAsync(q, w.out, abc::kPdQuantities * sizeof(float), hipMemcpyDeviceToHost, st));
    ABC_HIP(hipStreamSynchronize(st));
    energies_from(q, s, p, out);
    return ABC_OK;
}

int check_finite(const float* x, size_t n, const PdWs& w, hipStream_t st, const char* what) {
    ABC_HIP(hipMemsetAsync(w.flag, 0, sizeof(int), st));
    ABC_HIP(abc::launch_nonfinite(x, n, w.flag, st));
    int h = 0;
    ABC_HIP(hipMemcpyAsync(&h, w.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    ABC_HIP(hipStreamSynchronize(st));
    if (h) return fail(ABC_ENONFINITE, std::string(what) + " holds a NaN or Inf");
    return ABC_OK;
}

}  // namespace

namespace {
size_t tune_ws_bytes(int H, int W, int C);
int adjoint_dynamics_impl(const float* traj, int H, int W, int C, const float* eps, const abc_params* p,
                          const float* gK, float* g0, float* geps, void* ws, size_t ws_bytes, void* stream);

__global__ void zero_kernel(float* __restrict__ x, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0f;
}

__global__ void zero_i32_kernel(int* __restrict__ x, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0;
}

}  // namespace

// Scratch of abc_adjoint_dynamics_noalloc: one array per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, so the
// device address comes from hipGetSymbolAddress, once per device (with that
// device current), and only that address is handed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[ABC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_ptr(void** out) {
    int dev = 0;
    ABC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(ABC_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        ABC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(ABC_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return ABC_OK;
}
}

// ===========================================================================
extern "C" {

int abc_version(void) { return 100; }

int abc_support_radius(int H, int W, float eps_x_min, int32_t* R) {
    if (!R || H < 1 || W < 1 || !(eps_x_min >= 0.0f))
        return fail(ABC_EINVAL, "abc_support_radius: H, W >= 1, eps_x_min >= 0 and non-NULL R required");
    const int whole = std::max(H, W) - 1;
    const double r = std::ceil(std::sqrt(2.0 / (double)eps_x_min) * (double)std::max(H, W));
    *R = (eps_x_min == 0.0f || !(r < (double)whole)) ? whole : (int32_t)r;
    return ABC_OK;
}

const char* abc_last_error(void) { return g_last_error.c_str(); }

int abc_default_params(abc_params* p) {
    if (!p) return fail(ABC_EINVAL, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->K = 20;
    p->dt = 0.25f;
    p->R = 2;
    p->inv_norm = 0.0f;
    p->eps_min[0] = p->eps_min[1] = 2.0f;
    p->eps_max[0] = p->eps_max[1] = 1100.0f;
    p->eps_init = 57.0f;
    p->alpha = 3000.0f;
    p->rho = 1e-2f;
    p->gamma = 1e-2f;
    p->max_outer = 5;
    p->max_inner = 50;
    p->max_ls = 40;
    p->tol_alm = 0.0;
    p->tol_dal = 0.0;
    p->sigma0 = 1.0;
    p->armijo_b = 0.5;
    p->armijo_c = 1e-4;
    p->ckpt_every = 0;
    p->tile_x = p->tile_y = 0;
    return ABC_OK;
}

int abc_traj_slots(const abc_params* p, int* slots) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!slots) return fail(ABC_EINVAL, "slots is NULL");
    *slots = traj_slots(p);
    return ABC_OK;
}

int abc_workspace_bytes(int kind, int H, int W, int C, const abc_params* p, size_t* bytes) {
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_shape(H, W, C))) return rc;
    abc_params pr;
    p = with_radius(p, H, W, pr);
    if (!bytes) return fail(ABC_EINVAL, "bytes is NULL");
    if (kind < ABC_WS_SOLVE || kind > ABC_WS_TUNE) return fail(ABC_EINVAL, "unknown workspace kind");
    if (kind == ABC_WS_TUNE) {
        *bytes = tune_ws_bytes(H, W, C);
        return ABC_OK;
    }
    abc::Tile tf{32, 8}, ta{32, 8};
    if ((rc = pick_tile(p, C, 1, &tf))) return rc;
    if ((rc = pick_tile(p, C, 2, &ta))) return rc;
    *bytes = ws_bytes_for(kind, Shape{H, W, C}, p, tf, ta);
    return ABC_OK;
}

int abc_forward_dynamics(const float* c0, int H, int W, int C, const float* eps, const abc_params* p, float* traj,
                         void* ws, size_t ws_bytes, void* stream) {
    Range range("abc_forward_dynamics");
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_shape(H, W, C))) return rc;
    if (!c0 || !eps || !traj) return fail(ABC_EINVAL, "c0, eps and traj must be non-NULL");
    abc_params pr;
    p = with_radius(p, H, W, pr);
    const Shape s{H, W, C};
    abc::Tile t;
    if ((rc = pick_tile(p, C, 1, &t))) return rc;
    const size_t need = ws_bytes_for(ABC_WS_FORWARD, s, p, t, t);
    if (ws_bytes < need || (need > 0 && !ws)) return fail(ABC_EINVAL, "forward workspace too small");
    hipStream_t st = (hipStream_t)stream;
    const float dts = p->dt * norm_factor(p, s);
    if (p->ckpt_every <= 0) return forward_sweep_full(c0, traj, eps, s, p, dts, t, st);
    // checkpointed: slot m holds c^{min(m e, K)}; intermediate states ping-pong in ws
    const size_t f = s.field();
    Carve cv(ws);
    float* tmp[2] = {cv.take<float>(f), cv.take<float>(f)};
    ABC_HIP(hipMemcpyAsync(traj, c0, f * sizeof(float), hipMemcpyDeviceToDevice, st));
    const float* cur = traj;
    int slot = 1, flip = 0;
    for (int k = 0; k < p->K; ++k) {
        const bool at_ckpt = ((k + 1) % p->ckpt_every == 0) || (k + 1 == p->K);
        float* out = at_ckpt ? traj + (size_t)slot * f : tmp[flip];
        if (p->R == 0)
            ABC_HIP(hipMemcpyAsync(out, cur, f * sizeof(float), hipMemcpyDeviceToDevice, st));
        else
            ABC_HIP(abc::launch_forward_step(cur, out, eps, k, H, W, C, p->R, dts, t, st));
        cur = out;
        if (at_ckpt)
            ++slot;
        else
            flip ^= 1;
    }
    return ABC_OK;
}

int abc_adjoint_dynamics(const float* traj, int H, int W, int C, const float* eps, const abc_params* p,
                         const float* gK, float* g0, float* geps, void* ws, size_t ws_bytes, void* stream) {
    return adjoint_dynamics_impl(traj, H, W, C, eps, p, gK, g0, geps, ws, ws_bytes, stream);
}

int abc_adjoint_dynamics_noalloc(const float* traj, int H, int W, int C, const float* eps, const abc_params* p,
                                 const float* gK, float* g0, float* geps, void* stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_shape(H, W, C))) return rc;
    abc_params pr;
    p = with_radius(p, H, W, pr);
    abc::Tile tf, ta;
    if ((rc = pick_tile(p, C, 1, &tf))) return rc;
    if ((rc = pick_tile(p, C, 2, &ta))) return rc;
    const size_t need = ws_bytes_for(ABC_WS_ADJOINT, Shape{H, W, C}, p, tf, ta);
    if (need > ABC_NOALLOC_SCRATCH_BYTES)
        return fail(ABC_EINVAL, "abc_adjoint_dynamics_noalloc: this shape needs " + std::to_string(need) +
                                    " bytes of scratch, more than the " +
                                    std::to_string((size_t)ABC_NOALLOC_SCRATCH_BYTES) + " the library holds");
    void* sp = nullptr;
    if ((rc = scratch_ptr(&sp))) return rc;
    return adjoint_dynamics_impl(traj, H, W, C, eps, p, gK, g0, geps, sp, ABC_NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"

namespace {

int adjoint_dynamics_impl(const float* traj, int H, int W, int C, const float* eps, const abc_params* p,
                          const float* gK, float* g0, float* geps, void* ws, size_t ws_bytes, void* stream) {
    Range range("abc_adjoint_dynamics");
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_shape(H, W, C))) return rc;
    if (!traj || !eps || !gK || !g0 || !geps) return fail(ABC_EINVAL, "traj, eps, gK, g0, geps must be non-NULL");
    abc_params pr;
    p = with_radius(p, H, W, pr);
    const Shape s{H, W, C};
    abc::Tile tf, ta;
    if ((rc = pick_tile(p, C, 1, &tf))) return rc;
    if ((rc = pick_tile(p, C, 2, &ta))) return rc;
    const size_t need = ws_bytes_for(ABC_WS_ADJOINT, s, p, tf, ta);
    if (!ws || ws_bytes < need) return fail(ABC_EINVAL, "adjoint workspace too small");
    hipStream_t st = (hipStream_t)stream;
    const size_t f = s.field();
    const int tiles = abc::adj_part_count(H, W, C, p->R, ta);
    Carve cv(ws);
    AdjointWs w = carve_adjoint(cv, s, p, tiles);
    const float snorm = norm_factor(p, s);
    const float dts = p->dt * snorm;
    if (p->R == 0) {
        if (g0 != gK) ABC_HIP(hipMemcpyAsync(g0, gK, f * sizeof(float), hipMemcpyDeviceToDevice, st));
        // a kernel rather than a memset node, so that captured graphs replay it correctly
        const int n = p->K * 2;
        zero_kernel<<<(n + 255) / 256, 256, 0, st>>>(geps, n);
        ABC_HIP(hipGetLastError());
        return ABC_OK;
    }
    // The first step reads gK itself and the last one writes g0 itself (through the
    // ping-pong buffers in between), except that a single step with g0 == gK goes
    // through a buffer and a copy.
    const float* pin = gK;
    float* bufs[2] = {w.pa, w.pb};
    int nbuf = 0;
    auto step = [&](const float* ck, int k) -> int {
        float* out = (k == 0 && (const float*)g0 != pin) ? g0 : bufs[nbuf];
        ABC_HIP(abc::launch_adjoint_step(ck, pin, out, eps, k, s.H, s.W, s.C, p->R, dts, ta,
                                         w.part + (size_t)k * tiles * 2, st));
        if (out == bufs[nbuf]) nbuf ^= 1;
        pin = out;
        return ABC_OK;
    };
    if (p->ckpt_every <= 0) {
        for (int k = p->K - 1; k >= 0; --k)
            if ((rc = step(traj + (size_t)k * f, k))) return rc;
    } else {
        const int e = p->ckpt_every;
        const int nseg = (p->K + e - 1) / e;
        for (int m = nseg - 1; m >= 0; --m) {
            const int k0 = m * e, k1 = std::min(p->K, k0 + e);
            // recompute c^{k0+1..k1-1} from the checkpoint c^{k0} into the segment buffer
            std::vector<const float*> states(k1 - k0);
            states[0] = traj + (size_t)m * f;
            std::vector<float*> dst;
            for (int k = k0 + 1; k < k1; ++k) dst.push_back(w.seg + (size_t)(k - k0) * f);
            if (!dst.empty())
                if ((rc = forward_steps(states[0], dst.data(), k0, k1 - 1, eps, s, p, dts, tf, st))) return rc;
            for (int k = k0 + 1; k < k1; ++k) states[k - k0] = w.seg + (size_t)(k - k0) * f;
            for (int k = k1 - 1; k >= k0; --k)
                if ((rc = step(states[k - k0], k))) return rc;
        }
    }
    if (pin != g0) ABC_HIP(hipMemcpyAsync(g0, pin, f * sizeof(float), hipMemcpyDeviceToDevice, st));
    // dl/deps^k = -5 dt s * (raw sums of the adjoint kernel), summed in FP64
    ABC_HIP(abc::launch_reduce_rows_f64(w.part, p->K, tiles, 2, -5.0 * (double)p->dt * (double)snorm, nullptr, geps,
                                        st));
    return ABC_OK;
}

}  // namespace

extern "C" {

int abc_pd_terminal(const float* cK, const float* c0, const float* v, const float* mu, int H, int W, int C,
                    const abc_params* p, float* gK, double* Ltilde, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_shape(H, W, C))) return rc;
    if (!cK || !c0) return fail(ABC_EINVAL, "cK and c0 must be non-NULL");
    const Shape s{H, W, C};
    abc::Tile t{32, 8};
    const size_t need = ws_bytes_for(ABC_WS_PD, s, p, t, t);
    if (!ws || ws_bytes < need) return fail(ABC_EINVAL, "pd workspace too small");
    Carve cv(ws);
    PdWs w = carve_pd(cv, s);
    return objective(cK, c0, v, mu, gK, s, p, w, (hipStream_t)stream, Ltilde);
}

int abc_pd_step(const float* cK, const float* c0, int H, int W, int C, const abc_params* p, float* v, float* mu,
                int update_mu, abc_stats* st, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_shape(H, W, C))) return rc;
    if (!cK || !c0 || !v || !mu) return fail(ABC_EINVAL, "cK, c0, v and mu must be non-NULL");
    const Shape s{H, W, C};
    abc::Tile t{32, 8};
    const size_t need = ws_bytes_for(ABC_WS_PD, s, p, t, t);
    if (!ws || ws_bytes < need) return fail(ABC_EINVAL, "pd workspace too small");
    Carve cv(ws);
    PdWs w = carve_pd(cv, s);
    if (st) std::memset(st, 0, sizeof(*st));
    return pd_update(cK, c0, v, mu, update_mu, s, p, w, (hipStream_t)stream, st);
}

int abc_solve(const float* c0, int H, int W, int C, const abc_params* p, float* eps, float* mu, float* v_out,
              float* c_out, void* ws, size_t ws_bytes, void* stream, abc_stats* stats, abc_solve_log* log) {
    Range range("abc_solve");
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_shape(H, W, C))) return rc;
    abc_params pr;
    p = with_radius(p, H, W, pr);
    if (!c0 || !c_out) return fail(ABC_EINVAL, "c0 and c_out must be non-NULL");
    if (p->ckpt_every != 0) return fail(ABC_EINVAL, "abc_solve stores full trajectories; set ckpt_every = 0");
    const double* decisions_in = log ? log->decisions_in : nullptr;
    double* decisions_out = log ? log->decisions_out : nullptr;
    const double* eps_replay = log ? log->eps_replay : nullptr;
    double* grad_out = log ? log->grad_out : nullptr;
    double* phi_out = log ? log->phi_out : nullptr;
    double* outer_out = log ? log->outer_out : nullptr;
    double* eps_out = log ? log->eps_out : nullptr;
    if (eps_replay && !decisions_in) return fail(ABC_EINVAL, "eps_replay needs decisions_in");
    const auto t_start = std::chrono::steady_clock::now();
    const Shape s{H, W, C};
    abc::Tile tf, ta;
    if ((rc = pick_tile(p, C, 1, &tf))) return rc;
    if ((rc = pick_tile(p, C, 2, &ta))) return rc;
    const size_t need = ws_bytes_for(ABC_WS_SOLVE, s, p, tf, ta);
    if (!ws || ws_bytes < need) return fail(ABC_EINVAL, "solve workspace too small");
    hipStream_t st = (hipStream_t)stream;
    const int K = p->K;
    const size_t f = s.field();
    const int tiles = abc::adj_part_count(H, W, C, p->R, ta);
    Carve cv(ws);
    SolveWs w = carve_solve(cv, s, p, tiles);
    const float snorm = norm_factor(p, s);
    const float dts = p->dt * snorm;
    float* vv = v_out ? v_out : w.v;
    float* mm = mu ? mu : w.mu;
    const bool quad = p->cost == ABC_COST_QUADRATIC;
    abc_params pq = *p;  // parameters of the inner objective
    if (quad) pq.rho = 1.0f;

    if ((rc = check_finite(c0, f, w.pd, st, "input image"))) return rc;
    std::vector<double> e_base((size_t)K * 2), e_try((size_t)K * 2), e_cand((size_t)K * 2), e_next((size_t)K * 2);
    if (eps) {
        if ((rc = check_finite(eps, (size_t)K * 2, w.pd, st, "controls"))) return rc;
        std::vector<float> h((size_t)K * 2);
        ABC_HIP(hipMemcpyAsync(h.data(), eps, h.size() * sizeof(float), hipMemcpyDeviceToHost, st));
        ABC_HIP(hipStreamSynchronize(st));
        for (size_t i = 0; i < h.size(); ++i) e_base[i] = h[i];
    } else {
        std::fill(e_base.begin(), e_base.end(), (double)p->eps_init);
    }
    if (!mu || quad) ABC_HIP(hipMemsetAsync(mm, 0, 2 * f * sizeof(float), st));
    if (quad) ABC_HIP(hipMemsetAsync(vv, 0, 2 * f * sizeof(float), st));

    // Controls go up through a pinned staging array: the copy is queued without
    // a host wait, and every later upload comes after a host wait (the
    // objective read of the trial), so the array is free again by then.
    PinnedHost<float> stage;
    stage.st = st;
    if ((rc = stage.alloc((size_t)K * 2))) return rc;
    // the control gradient comes back through a pinned array too (read after the wait below)
    PinnedHost<double> gstage;
    gstage.st = st;
    if ((rc = gstage.alloc((size_t)K * 2))) return rc;
    auto upload = [&](const std::vector<double>& e, float* dev) -> int {
        for (size_t i = 0; i < e.size(); ++i) stage.ptr[i] = (float)e[i];
        ABC_HIP(hipMemcpyAsync(dev, stage.ptr, e.size() * sizeof(float), hipMemcpyHostToDevice, st));
        return ABC_OK;
    };
    auto project = [&](const std::vector<double>& G, double tau, std::vector<double>& out) {
        for (int k = 0; k < K; ++k)
            for (int m = 0; m < 2; ++m) {
                const double x = e_base[2 * k + m] - tau * G[2 * k + m];
                out[2 * k + m] = std::min<double>(std::max<double>(x, p->eps_min[m]), p->eps_max[m]);
            }
    };
    const size_t traj_stride = (size_t)K * f;  // offset of c^K inside a trajectory
    int base = 0, cand = 1, trial = 2;
    GraphCache& graphs = solve_graphs();
    const bool use_graphs = !(p->flags & ABC_FLAG_NO_GRAPHS) && p->R > 0;
    // what the recorded sweeps depend on: device, workspace (every buffer is carved
    // from it in a fixed order), sizes, window, launch shapes and the step scale
    int device = 0;
    ABC_HIP(hipGetDevice(&device));
    auto gkey = [&](long kind, long idx) -> std::vector<long> {
        return {kind, idx, (long)device, (long)(uintptr_t)ws, (long)H, (long)W, (long)C, (long)K, (long)p->R,
                float_bits(dts), float_bits(snorm), (long)tf.tx, (long)tf.ty, (long)ta.tx, (long)ta.ty};
    };
    // slot 0 of every trajectory holds c0 for the whole solve
    for (int b = 0; b < 3; ++b) ABC_HIP(hipMemcpyAsync(w.traj[b], c0, f * sizeof(float), hipMemcpyDeviceToDevice, st));
    // K forward steps into trajectory buffer `idx` under the controls eps[idx]
    auto sweep = [&](int idx) -> int {
        if (p->R == 0) return forward_sweep_full(c0, w.traj[idx], w.eps[idx], s, p, dts, tf, st);
        return graphs.run(use_graphs, gkey(0, idx), st, [&](hipStream_t s2) -> int {
            for (int k = 0; k < K; ++k)
                ABC_HIP(abc::launch_forward_step(w.traj[idx] + k * f, w.traj[idx] + (k + 1) * f, w.eps[idx], k, H, W, C,
                                                 p->R, dts, tf, s2));
            return ABC_OK;
        });
    };
    // Armijo trial into buffer `trial`: eps(tau), forward sweep, Phi(tau), test.
    double K_try = 0.0;  // TV energy of the last trial's final field
    auto run_trial = [&](const std::vector<double>& G, double tau, double phi0, double* phit, bool* ok) -> int {
        Range trial_range("Armijo trial");
        project(G, tau, e_try);
        int r2 = upload(e_try, w.eps[trial]);
        if (r2) return r2;
        if ((r2 = sweep(trial))) return r2;
        if ((r2 = objective(w.traj[trial] + traj_stride, c0, vv, mm, nullptr, s, &pq, w.pd, st, phit, &K_try)))
            return r2;
        double ip = 0.0;
        for (int i = 0; i < 2 * K; ++i) ip += G[i] * (e_try[i] - e_base[i]);
        ip *= (double)p->dt;
        *ok = *phit <= phi0 + p->armijo_c * ip;
        return ABC_OK;
    };

    abc_stats S;
    std::memset(&S, 0, sizeof(S));
    S.gap_rel = NAN;
    const int M = p->max_outer, P = p->max_inner;
    const size_t nslots = (size_t)M * P;
    if (decisions_out) std::fill(decisions_out, decisions_out + nslots, 0.0);
    if (grad_out) std::fill(grad_out, grad_out + nslots * 2 * K, 0.0);
    if (phi_out) std::fill(phi_out, phi_out + nslots * kStepLog, 0.0);
    if (outer_out) std::fill(outer_out, outer_out + (size_t)M * 4, 0.0);
    if (eps_out) std::fill(eps_out, eps_out + nslots * 2 * K, 0.0);

    // Alg. 2: forward integration, v^(0) = argmin_v L(c^(0), v, mu^(0)).
    if ((rc = upload(e_base, w.eps[base]))) return rc;
    if ((rc = sweep(base))) return rc;
    abc_stats E0;
    std::memset(&E0, 0, sizeof(E0));
    const bool check0 = !quad && p->stop_K > 0.0;
    if (!quad && (rc = pd_update(w.traj[base] + traj_stride, c0, vv, mm, 0, s, p, w.pd, st, check0 ? &E0 : nullptr)))
        return rc;
    // energy target already met by the starting controls (e.g. a warm start): no iteration needed
    const bool done0 = check0 && E0.K <= p->stop_K;
    const double ms_start = ms_since(t_start);

    double sigma = p->sigma0;
    double L_prev = NAN;
    bool phi_seen = false;
    abc_stats E;
    std::memset(&E, 0, sizeof(E));
    std::vector<double> G;
    double K_acc = 0.0;  // TV energy after the last accepted step
    bool hit_K = false;
    const int n_outer = quad ? std::min(M, 1) : (done0 ? 0 : M);
    if (done0) E = E0;
    for (int j = 0; j < n_outer; ++j) {
        Range outer_range("multiplier iteration");
        for (int it = 0; it < P; ++it) {
            Range inner_range("DAL iteration");
            const size_t slot = (size_t)j * P + it;
            // terminal condition and objective at the accepted controls, queued; read
            // together with the control gradient after the adjoint sweep
            double phi0 = 0.0;
            ABC_HIP(abc::launch_terminal(w.traj[base] + traj_stride, c0, vv, mm, H, W, C, pq.rho, pq.alpha,
                                         (float)s.area(), w.adj.pa, w.pd.part, st));
            ABC_HIP(abc::launch_reduce_rows(w.pd.part, 1, abc::pd_blocks(H, W), abc::kTermQuantities, w.pd.out, 1.0f,
                                            st));
            // adjoint sweep from p^K = dL~/dc, then the control gradient
            float* cur = w.adj.pa;
            float* spare = w.adj.pb;
            if (p->R > 0) {
                std::vector<const float*> states(K);
                for (int k = 0; k < K; ++k) states[k] = w.traj[base] + (size_t)k * f;
                rc = graphs.run(use_graphs, gkey(1, base), st, [&](hipStream_t s2) -> int {
                    float* c2 = cur;
                    float* sp2 = spare;
                    int r3 = adjoint_steps(states.data(), 0, K, w.eps[base], s, p, dts, ta, c2, sp2, w.adj.part, tiles,
                                           s2);
                    if (r3) return r3;
                    ABC_HIP(abc::launch_reduce_rows_f64(w.adj.part, K, tiles, 2, -5.0 * (double)snorm, w.G, nullptr,
                                                        s2));
                    return ABC_OK;
                });
                if (rc) return rc;
                G.resize((size_t)K * 2);
                ABC_HIP(hipMemcpyAsync(gstage.ptr, w.G, G.size() * sizeof(double), hipMemcpyDeviceToHost, st));
            } else {
                G.assign((size_t)K * 2, 0.0);
            }
            {
                float local[abc::kTermQuantities];
                float* h = scalar_readback();
                if (!h) h = local;
                ABC_HIP(hipMemcpyAsync(h, w.pd.out, abc::kTermQuantities * sizeof(float), hipMemcpyDeviceToHost, st));
                ABC_HIP(hipStreamSynchronize(st));
                phi0 = s.area() * (double)h[0];
                if (p->R > 0) std::copy(gstage.ptr, gstage.ptr + G.size(), G.begin());
            }
            if (!phi_seen) {
                S.phi_first = phi0;
                phi_seen = true;
            }
            S.phi_last = phi0;
            S.inner_iters++;
            if (grad_out) std::copy(G.begin(), G.end(), grad_out + slot * 2 * K);
            if (phi_out) phi_out[kStepLog * slot] = phi0;
            bool all_zero = true;
            for (double g : G) all_zero = all_zero && (g == 0.0);
            if (decisions_in && !(decisions_in[slot] > 0.0)) break;
            if (!decisions_in && all_zero) break;

            double accepted = 0.0, phi_acc = phi0;
            if (decisions_in) {
                accepted = decisions_in[slot];
                bool ok = false;
                if (eps_replay) {
                    // the step this iteration's own gradient gives, logged but not taken
                    if (eps_out) {
                        project(G, accepted, e_next);
                        std::copy(e_next.begin(), e_next.end(), eps_out + slot * 2 * K);
                    }
                    e_try.assign(eps_replay + slot * 2 * K, eps_replay + (slot + 1) * 2 * K);
                    if ((rc = upload(e_try, w.eps[trial]))) return rc;
                    if ((rc = sweep(trial))) return rc;
                    if ((rc = objective(w.traj[trial] + traj_stride, c0, vv, mm, nullptr, s, &pq, w.pd, st, &phi_acc,
                                        &K_try)))
                        return rc;
                } else if ((rc = run_trial(G, accepted, phi0, &phi_acc, &ok))) {
                    return rc;
                }
                std::swap(cand, trial);
                e_cand = e_try;
                K_acc = K_try;
                S.ls_evals++;
                if (phi_out) phi_out[kStepLog * slot + 2] = 1;
            } else {
                double tau = sigma, phit = 0.0;
                bool ok = false, have = false;
                int evals = 0;
                if ((rc = run_trial(G, tau, phi0, &phit, &ok))) return rc;
                evals++;
                if (ok) {
                    // expanding branch
                    std::swap(cand, trial);
                    e_cand = e_try;
                    accepted = tau;
                    phi_acc = phit;
                    K_acc = K_try;
                    have = true;
                    while (evals < p->max_ls) {
                        project(G, tau / p->armijo_b, e_next);
                        if (e_next == e_cand) break;  // the projected point no longer moves
                        tau /= p->armijo_b;
                        if ((rc = run_trial(G, tau, phi0, &phit, &ok))) return rc;
                        evals++;
                        if (!ok) break;
                        std::swap(cand, trial);
                        e_cand = e_try;
                        accepted = tau;
                        phi_acc = phit;
                        K_acc = K_try;
                    }
                } else {
                    // backtracking branch
                    while (evals < p->max_ls) {
                        tau *= p->armijo_b;
                        if ((rc = run_trial(G, tau, phi0, &phit, &ok))) return rc;
                        evals++;
                        if (ok) {
                            std::swap(cand, trial);
                            e_cand = e_try;
                            accepted = tau;
                            phi_acc = phit;
                            K_acc = K_try;
                            have = true;
                            break;
                        }
                    }
                }
                S.ls_evals += evals;
                if (phi_out) phi_out[kStepLog * slot + 2] = evals;
                if (!have) break;
                sigma = accepted;
            }
            e_base = e_cand;
            std::swap(base, cand);
            if (decisions_out) decisions_out[slot] = accepted;
            if (eps_out && !eps_replay) std::copy(e_base.begin(), e_base.end(), eps_out + slot * 2 * K);
            if (phi_out) {
                phi_out[kStepLog * slot + 1] = phi_acc;
                phi_out[kStepLog * slot + 3] = K_acc;
                phi_out[kStepLog * slot + 4] = ms_since(t_start);
            }
            if (!quad && p->stop_K > 0.0 && K_acc <= p->stop_K) {
                hit_K = true;  // energy target met by this step: no further iteration
                break;
            }
            if (p->tol_dal > 0.0 && std::fabs(phi_acc - phi0) < p->tol_dal * std::fabs(phi0)) break;
        }
        if (hit_K) {
            S.outer_iters = j + 1;
            break;
        }
        if (quad) {
            S.outer_iters = 1;
            break;
        }
        // v- and mu-updates (eq. soft_threshold, eq. dual_ascent)
        if ((rc = pd_update(w.traj[base] + traj_stride, c0, vv, mm, 1, s, p, w.pd, st, &E))) return rc;
        S.outer_iters = j + 1;
        S.gap_rel = std::isnan(L_prev) ? NAN : std::fabs(E.L - L_prev) / std::fabs(L_prev);
        L_prev = E.L;
        if (outer_out) {
            outer_out[4 * j + 0] = E.K;
            outer_out[4 * j + 1] = E.L;
            outer_out[4 * j + 2] = E.r_rel;
            outer_out[4 * j + 3] = ms_since(t_start);
        }
        if (p->tol_alm > 0.0 && E.r_rel < p->tol_alm) break;
        if (p->stop_K > 0.0 && E.K <= p->stop_K) break;
        // the change of the Lagrangian between multiplier iterations is small (Sec. 4.1)
        if (p->tol_gap > 0.0 && !std::isnan(S.gap_rel) && S.gap_rel < p->tol_gap) break;
    }
    if (quad) {
        // TV and fidelity of the final field from the pd kernel on scratch copies (v, mu stay 0);
        // the inner objective is J itself
        // the two spare trajectories are free here and each holds at least 2 fields (K >= 1)
        float* sv = w.traj[trial];
        float* sm = w.traj[cand];
        ABC_HIP(hipMemsetAsync(sv, 0, 2 * f * sizeof(float), st));
        ABC_HIP(hipMemsetAsync(sm, 0, 2 * f * sizeof(float), st));
        if ((rc = pd_update(w.traj[base] + traj_stride, c0, sv, sm, 0, s, p, w.pd, st, &E))) return rc;
        double J = 0.0;
        if ((rc = objective(w.traj[base] + traj_stride, c0, vv, mm, nullptr, s, &pq, w.pd, st, &J))) return rc;
        E.L = E.Ltilde = J;
        E.r_rel = E.r_abs = 0.0;
    } else if (hit_K) {
        // energies of the final field with its v-argmin (computed on a spare buffer; mu unchanged)
        if ((rc = pd_update(w.traj[base] + traj_stride, c0, w.traj[trial], mm, 0, s, p, w.pd, st, &E))) return rc;
    } else if (S.outer_iters == 0 && !done0) {
        // no multiplier step taken: energies at the initial state (v is unchanged by this call)
        if ((rc = pd_update(w.traj[base] + traj_stride, c0, vv, mm, 0, s, p, w.pd, st, &E))) return rc;
    }
    ABC_HIP(hipMemcpyAsync(c_out, w.traj[base] + traj_stride, f * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (eps) {
        std::vector<float> h(e_base.size());
        for (size_t i = 0; i < h.size(); ++i) h[i] = (float)e_base[i];
        ABC_HIP(hipMemcpyAsync(eps, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, st));
    }
    ABC_HIP(hipStreamSynchronize(st));
    S.K = E.K;
    S.TV = E.TV;
    S.fid = E.fid;
    S.L = E.L;
    S.Ltilde = E.Ltilde;
    S.r_rel = E.r_rel;
    S.r_abs = E.r_abs;
    S.status = (!quad && p->tol_alm > 0.0 && !(E.r_rel < p->tol_alm)) ? ABC_ENOCONV : ABC_OK;
    S.K_start = check0 ? E0.K : NAN;
    S.ms_start = ms_start;
    if (stats) *stats = S;
    return S.status;
}

}  // extern "C"

namespace {

struct TuneEntry {
    int ftx, fty, atx, aty;
    double fus, aus;
};

std::map<std::string, TuneEntry> read_tune_cache(const char* path) {
    std::map<std::string, TuneEntry> out;
    if (!path) return out;
    FILE* fp = std::fopen(path, "r");
    if (!fp) return out;
    char line[1024];
    while (std::fgets(line, sizeof(line), fp)) {
        const char* q1 = std::strchr(line, '"');
        if (!q1) continue;
        const char* q2 = std::strchr(q1 + 1, '"');
        if (!q2) continue;
        TuneEntry e;
        if (std::sscanf(q2 + 1, ": {\"fwd\": [%d, %d], \"adj\": [%d, %d], \"fwd_us\": %lf, \"adj_us\": %lf}", &e.ftx,
                        &e.fty, &e.atx, &e.aty, &e.fus, &e.aus) == 6)
            out[std::string(q1 + 1, q2)] = e;
    }
    std::fclose(fp);
    return out;
}

bool write_tune_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return false;
    std::fprintf(fp, "{\n");
    size_t i = 0;
    for (const auto& kv : m) {
        const TuneEntry& e = kv.second;
        std::fprintf(fp, "  \"%s\": {\"fwd\": [%d, %d], \"adj\": [%d, %d], \"fwd_us\": %.3f, \"adj_us\": %.3f}%s\n",
                     kv.first.c_str(), e.ftx, e.fty, e.atx, e.aty, e.fus, e.aus, (++i < m.size()) ? "," : "");
    }
    std::fprintf(fp, "}\n");
    std::fclose(fp);
    return std::rename(tmp.c_str(), path) == 0;
}

const abc::Tile kTuneCands[] = {{32, 16}, {64, 8}, {16, 32}, {128, 4}, {32, 8}, {16, 16}, {64, 4}, {128, 2},
                                {16, 8},  {32, 4}, {64, 2},  {8, 16},  {8, 8},  {16, 4},  {32, 2}, {64, 1}};

size_t tune_ws_bytes(int H, int W, int C) {
    Carve cv(nullptr);
    const size_t f = (size_t)H * W * C;
    cv.take<float>(f);
    cv.take<float>(f);
    cv.take<float>(2);
    int maxt = 0;
    for (const abc::Tile& t : kTuneCands) maxt = std::max(maxt, abc::tile_count(H, W, t));
    cv.take<double>((size_t)maxt * 2);
    return cv.used;
}


// Times the forward and adjoint interaction kernels on c0 for every admissible
// tile shape and returns the fastest of each in *best.  ws: tune_ws_bytes().
int tune_tiles(const float* c0, int H, int W, int C, const abc_params* p, void* ws, hipStream_t st, TuneEntry* best) {
    const size_t f = (size_t)H * W * C;
    Carve cv(ws);
    float* out = cv.take<float>(f);
    float* pout = cv.take<float>(f);
    float* eps = cv.take<float>(2);
    double* part = nullptr;
    {
        int maxt = 0;
        for (const abc::Tile& t : kTuneCands) maxt = std::max(maxt, abc::tile_count(H, W, t));
        part = cv.take<double>((size_t)maxt * 2);
    }
    const float e2[2] = {p->eps_init, p->eps_init};
    ABC_HIP(hipMemcpyAsync(eps, e2, sizeof(e2), hipMemcpyHostToDevice, st));
    ABC_HIP(hipStreamSynchronize(st));
    const Shape s{H, W, C};
    const float dts = p->dt * norm_factor(p, s);
    hipEvent_t ev0, ev1;
    ABC_HIP(hipEventCreate(&ev0));
    ABC_HIP(hipEventCreate(&ev1));
    *best = TuneEntry{0, 0, 0, 0, 1e30, 1e30};
    constexpr int kReps = 5;
    int rc = ABC_OK;
    for (int kind = 0; kind < 2 && rc == ABC_OK; ++kind) {
        for (const abc::Tile& t : kTuneCands) {
            if (!abc::tile_ok(C, p->R, t, kind + 1)) continue;
            auto launch = [&]() -> hipError_t {
                return kind == 0 ? abc::launch_forward_step(c0, out, eps, 0, H, W, C, p->R, dts, t, st)
                                 : abc::launch_adjoint_step(c0, c0, pout, eps, 0, H, W, C, p->R, dts, t, part, st);
            };
            hipError_t e = launch();  // warm-up (also sets the LDS attribute)
            if (e != hipSuccess) continue;
            float ms_best = 1e30f;
            for (int rep = 0; rep < 3 && rc == ABC_OK; ++rep) {
                hipError_t e1 = hipEventRecord(ev0, st);
                for (int i = 0; i < kReps && e1 == hipSuccess; ++i) e1 = launch();
                if (e1 == hipSuccess) e1 = hipEventRecord(ev1, st);
                if (e1 == hipSuccess) e1 = hipEventSynchronize(ev1);
                float ms = 0.0f;
                if (e1 == hipSuccess) e1 = hipEventElapsedTime(&ms, ev0, ev1);
                if (e1 != hipSuccess) {
                    rc = fail(ABC_EHIP, std::string("autotune timing: ") + hipGetErrorString(e1));
                    break;
                }
                ms_best = std::min(ms_best, ms);
            }
            if (rc) break;
            const double us = 1e3 * (double)ms_best / kReps;
            if (kind == 0 && us < best->fus) *best = TuneEntry{t.tx, t.ty, best->atx, best->aty, us, best->aus};
            if (kind == 1 && us < best->aus) *best = TuneEntry{best->ftx, best->fty, t.tx, t.ty, best->fus, us};
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (rc) return rc;
    if (best->ftx == 0 || best->atx == 0)
        return fail(ABC_EINVAL, "no admissible tile for this channel count and radius");
    return ABC_OK;
}

std::string gpu_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string arch(prop.gcnArchName);
    return arch.substr(0, arch.find(':'));
}

}  // namespace

// ===========================================================================
// Batched solve: lockstep rounds over many images of different sizes.
namespace {

// Where an image of a batched solve stands: it needs a gradient (objective
// and adjoint sweep at its accepted controls), the next Armijo trial, its
// multiplier update, or nothing more.
constexpr int kPhGrad = 0, kPhSearch = 1, kPhPd = 2, kPhDone = 3;

struct BImg {
    // geometry
    int H, W;
    size_t f;
    int tiles_f, tiles_a, pdb;
    float snorm, dts;
    double area;
    // device buffers
    float* traj[3];
    float* pa;
    float* pb;
    double* gpart;
    float* v;
    float* mu;
    float* pdpart;
    // caller's arrays
    const float* c0;
    float* c_out;
    float* eps_user;
    float* mu_user;
    // host state
    std::vector<double> e_base, e_try, e_cand, e_next, G;
    double sigma = 0, phi0 = 0, phi_acc = 0, accepted = 0, tau = 0, L_prev = NAN;
    int base = 0, cand = 1, trial = 2;
    int evals = 0, branch = 0;  // 0: first trial, 1: expanding, 2: backtracking
    bool have = false, outer_done = false, ls_done = false, phi_seen = false;
    int phase = 0;  // kPhGrad, kPhSearch, kPhPd or kPhDone
    int j = 0;      // multiplier iteration in progress
    int it = 0;     // gradient evaluations within it
    double K_acc = 0.0;             // TV energy after the last accepted trial
    const abc_solve_log* log = nullptr;  // caller's record / replay arrays (may be NULL)
    abc_stats S;
    abc_stats E;
    double finish_ms = 0;
};

// Job tables and reduction outputs of one launch stream.
struct BatchLane {
    abc::StepJob* step_jobs;
    abc::PixJob* pix_jobs;
    abc::RedJob* red_jobs;
    float* q_all;  // n x kPdQuantities
    int* queue;    // K x 8 tile counters of the persistent sweeps
    hipStream_t st;
};

struct BatchWs {
    BatchLane a, b;    // a: gradients and multiplier updates, b: Armijo trials
    float* eps_all;    // n x 3 x K x 2
    double* g_all;     // n x K x 2
};

void carve_batch(Carve& cv, int n, int K, BatchWs& b) {
    for (BatchLane* l : {&b.a, &b.b}) {
        l->step_jobs = cv.take<abc::StepJob>(n);
        l->pix_jobs = cv.take<abc::PixJob>(n);
        l->red_jobs = cv.take<abc::RedJob>(n);
        l->q_all = cv.take<float>((size_t)n * abc::kPdQuantities);
        l->queue = cv.take<int>((size_t)K * 8);
        l->st = nullptr;
    }
    b.eps_all = cv.take<float>((size_t)n * 3 * K * 2);
    b.g_all = cv.take<double>((size_t)n * K * 2);
}

void carve_bimg(Carve& cv, BImg& m, int K, int C) {
    for (int i = 0; i < 3; ++i) m.traj[i] = cv.take<float>((size_t)(K + 1) * m.f);
    m.pa = cv.take<float>(m.f);
    m.pb = cv.take<float>(m.f);
    m.gpart = cv.take<double>((size_t)K * m.tiles_a * 2);
    m.v = cv.take<float>(2 * m.f);
    m.mu = cv.take<float>(2 * m.f);
    m.pdpart = cv.take<float>((size_t)m.pdb * abc::kPdQuantities);
    (void)C;
}

struct Batch {
    int n, C, K;
    const abc_params* p;
    abc_params pq;  // inner-objective parameters (rho = 1 for the quadratic cost)
    bool quad;
    abc::Tile tf, ta;
    hipStream_t st;
    bool use_graphs = false;
    std::vector<BImg> im;
    BatchWs w;
    std::vector<float> eps_host;  // mirror of eps_all
    GraphCache graphs;
    bool persistent = false;      // sweeps as persistent launches over per-step tile queues
    hipStream_t own_b = nullptr;  // lane b's stream, created for the call

    Batch() = default;
    Batch(const Batch&) = delete;
    Batch& operator=(const Batch&) = delete;
    ~Batch() {
        if (own_b) {
            (void)hipStreamSynchronize(own_b);
            (void)hipStreamDestroy(own_b);
        }
    }

    float* eps_dev(int i, int slot) const { return w.eps_all + ((size_t)i * 3 + slot) * K * 2; }

    int upload_eps(const std::vector<int>& who, const std::vector<int>& slot,
                   const std::vector<const std::vector<double>*>& vals, hipStream_t s) {
        for (size_t j = 0; j < who.size(); ++j) {
            float* h = eps_host.data() + ((size_t)who[j] * 3 + slot[j]) * K * 2;
            for (int q = 0; q < 2 * K; ++q) h[q] = (float)(*vals[j])[q];
        }
        // the whole mirror: entries of images not listed are rewritten with the values they hold
        ABC_HIP(hipMemcpyAsync(w.eps_all, eps_host.data(), eps_host.size() * sizeof(float), hipMemcpyHostToDevice,
                               s));
        return ABC_OK;
    }

    // K forward steps of every listed image into its trajectory `slot[j]`.
    int forward(const std::vector<int>& who, const std::vector<int>& slot, BatchLane& L) {
        hipStream_t st = L.st;
        if (who.empty()) return ABC_OK;
        std::vector<abc::StepJob> jobs(who.size());
        int total = 0;
        for (size_t j = 0; j < who.size(); ++j) {
            const BImg& m = im[who[j]];
            abc::StepJob& J = jobs[j];
            std::memset(&J, 0, sizeof(J));
            J.traj = m.traj[slot[j]];
            J.eps = eps_dev(who[j], slot[j]);
            J.H = m.H;
            J.W = m.W;
            J.tiles_x = (m.W + tf.tx - 1) / tf.tx;
            J.tiles = m.tiles_f;
            J.start = total;
            J.dts = m.dts;
            J.dx2 = 1.0f / ((float)m.W * (float)m.W);
            J.dy2 = 1.0f / ((float)m.H * (float)m.H);
            total += m.tiles_f;
        }
        ABC_HIP(hipMemcpyAsync(L.step_jobs, jobs.data(), jobs.size() * sizeof(abc::StepJob), hipMemcpyHostToDevice,
                               st));
        if (p->R == 0) {
            for (int k = 0; k < K; ++k)
                for (size_t j = 0; j < who.size(); ++j) {
                    const BImg& m = im[who[j]];
                    float* t = m.traj[slot[j]];
                    ABC_HIP(hipMemcpyAsync(t + (size_t)(k + 1) * m.f, t, m.f * sizeof(float), hipMemcpyDeviceToDevice,
                                           st));
                }
            return ABC_OK;
        }
        const int nj = (int)jobs.size();
        // a recorded sweep reads the lane's own job table, so the lane is part of the key
        const long lane = &L == &w.b ? 1 : 0;
        return graphs.run(use_graphs, {0, total, nj, lane}, st, [&](hipStream_t s2) -> int {
            int* q = persistent ? L.queue : nullptr;
            if (q) {
                zero_i32_kernel<<<(K * 8 + 255) / 256, 256, 0, s2>>>(q, K * 8);
                ABC_HIP(hipGetLastError());
            }
            for (int k = 0; k < K; ++k)
                ABC_HIP(abc::launch_forward_step_batched(L.step_jobs, nj, total, k, C, p->R, tf, q, s2));
            return ABC_OK;
        });
    }

    // Terminal condition (into pa) and/or objective of trajectory `slot[j]`, queued on the lane.
    int objective_launch(const std::vector<int>& who, const std::vector<int>& slot, bool want_pK, BatchLane& L) {
        if (who.empty()) return ABC_OK;
        hipStream_t st = L.st;
        std::vector<abc::PixJob> jobs(who.size());
        std::vector<abc::RedJob> reds(who.size());
        int total = 0;
        for (size_t j = 0; j < who.size(); ++j) {
            const BImg& m = im[who[j]];
            abc::PixJob& J = jobs[j];
            J.c = m.traj[slot[j]] + (size_t)K * m.f;
            J.c0 = m.c0;
            J.v = m.v;
            J.mu = m.mu;
            J.pK = want_pK ? m.pa : nullptr;
            J.part = m.pdpart;
            J.H = m.H;
            J.W = m.W;
            J.start = total;
            J.area = (float)m.area;
            J.inv2dx = 0.5f * (float)m.W;
            J.inv2dy = 0.5f * (float)m.H;
            total += m.pdb;
            abc::RedJob& Rj = reds[j];
            std::memset(&Rj, 0, sizeof(Rj));
            Rj.part_f = m.pdpart;
            Rj.out_f = L.q_all + (size_t)j * abc::kPdQuantities;
            Rj.rows = 1;
            Rj.nblk = m.pdb;
        }
        ABC_HIP(hipMemcpyAsync(L.pix_jobs, jobs.data(), jobs.size() * sizeof(abc::PixJob), hipMemcpyHostToDevice, st));
        ABC_HIP(hipMemcpyAsync(L.red_jobs, reds.data(), reds.size() * sizeof(abc::RedJob), hipMemcpyHostToDevice, st));
        ABC_HIP(abc::launch_terminal_batched(L.pix_jobs, (int)jobs.size(), total, C, pq.rho, pq.alpha, st));
        ABC_HIP(abc::launch_reduce_jobs(L.red_jobs, (int)reds.size(), abc::kTermQuantities, st));
        return ABC_OK;
    }

    // Waits for the lane and reads the objectives queued by objective_launch into
    // phi (and the TV energies K = TV + fidelity of the same fields into Kv, if given).
    int objective_read(const std::vector<int>& who, BatchLane& L, std::vector<double>& phi,
                       std::vector<double>* Kv = nullptr) {
        phi.assign(who.size(), 0.0);
        if (Kv) Kv->assign(who.size(), 0.0);
        if (who.empty()) return ABC_OK;
        std::vector<float> q(who.size() * abc::kPdQuantities);
        ABC_HIP(hipMemcpyAsync(q.data(), L.q_all, q.size() * sizeof(float), hipMemcpyDeviceToHost, L.st));
        ABC_HIP(hipStreamSynchronize(L.st));
        for (size_t j = 0; j < who.size(); ++j) {
            const double a = im[who[j]].area;
            const float* qj = q.data() + j * abc::kPdQuantities;
            phi[j] = a * (double)qj[0];
            if (Kv) (*Kv)[j] = a * (double)qj[1] + a * 0.5 * (double)p->alpha * (double)qj[2];
        }
        return ABC_OK;
    }

    int objective(const std::vector<int>& who, const std::vector<int>& slot, bool want_pK, std::vector<double>& phi,
                  BatchLane& L) {
        int rc = objective_launch(who, slot, want_pK, L);
        return rc ? rc : objective_read(who, L, phi);
    }

    // Adjoint sweep from p^K (in pa) over each image's base trajectory; fills G.
    int adjoint(const std::vector<int>& who) {
        if (who.empty()) return ABC_OK;
        BatchLane& L = w.a;
        hipStream_t st = L.st;
        std::vector<abc::StepJob> jobs(who.size());
        std::vector<abc::RedJob> reds(who.size());
        int total = 0;
        for (size_t j = 0; j < who.size(); ++j) {
            BImg& m = im[who[j]];
            abc::StepJob& J = jobs[j];
            J.traj = m.traj[m.base];
            J.eps = eps_dev(who[j], m.base);
            J.pa = m.pa;
            J.pb = m.pb;
            J.part = m.gpart;
            J.H = m.H;
            J.W = m.W;
            J.tiles_x = (m.W + ta.tx - 1) / ta.tx;
            J.tiles = m.tiles_a;
            J.start = total;
            J.dts = m.dts;
            J.dx2 = 1.0f / ((float)m.W * (float)m.W);
            J.dy2 = 1.0f / ((float)m.H * (float)m.H);
            total += m.tiles_a;
            abc::RedJob& Rj = reds[j];
            std::memset(&Rj, 0, sizeof(Rj));
            Rj.part_d = m.gpart;
            Rj.out_d = w.g_all + (size_t)j * K * 2;
            Rj.scale = -5.0 * (double)m.snorm;
            Rj.rows = K;
            Rj.nblk = m.tiles_a;
        }
        if (p->R > 0) {
            ABC_HIP(hipMemcpyAsync(L.step_jobs, jobs.data(), jobs.size() * sizeof(abc::StepJob),
                                   hipMemcpyHostToDevice, st));
            ABC_HIP(hipMemcpyAsync(L.red_jobs, reds.data(), reds.size() * sizeof(abc::RedJob), hipMemcpyHostToDevice,
                                   st));
            const int nj = (int)jobs.size();
            int r2 = graphs.run(use_graphs, {1, total, nj, 0}, st, [&](hipStream_t s2) -> int {
                int* q = persistent ? L.queue : nullptr;
                if (q) {
                    zero_i32_kernel<<<(K * 8 + 255) / 256, 256, 0, s2>>>(q, K * 8);
                    ABC_HIP(hipGetLastError());
                }
                for (int k = K - 1; k >= 0; --k)
                    ABC_HIP(abc::launch_adjoint_step_batched(L.step_jobs, nj, total, k, K, C, p->R, ta, q, s2));
                ABC_HIP(abc::launch_reduce_jobs_f64(L.red_jobs, nj, K, 2, s2));
                return ABC_OK;
            });
            if (r2) return r2;
            std::vector<double> g(who.size() * K * 2);
            ABC_HIP(hipMemcpyAsync(g.data(), w.g_all, g.size() * sizeof(double), hipMemcpyDeviceToHost, st));
            ABC_HIP(hipStreamSynchronize(st));
            for (size_t j = 0; j < who.size(); ++j)
                im[who[j]].G.assign(g.begin() + j * K * 2, g.begin() + (j + 1) * K * 2);
        } else {
            for (int i : who) im[i].G.assign((size_t)K * 2, 0.0);
        }
        return ABC_OK;
    }

    // Shrinkage / multiplier update of each listed image's final field; energies into E.
    int pd(const std::vector<int>& who, int update_mu, bool want) {
        if (who.empty()) return ABC_OK;
        BatchLane& L = w.a;
        hipStream_t st = L.st;
        std::vector<abc::PixJob> jobs(who.size());
        std::vector<abc::RedJob> reds(who.size());
        int total = 0;
        for (size_t j = 0; j < who.size(); ++j) {
            const BImg& m = im[who[j]];
            abc::PixJob& J = jobs[j];
            std::memset(&J, 0, sizeof(J));
            J.c = m.traj[m.base] + (size_t)K * m.f;
            J.c0 = m.c0;
            J.v = m.v;
            J.mu = m.mu;
            J.part = m.pdpart;
            J.H = m.H;
            J.W = m.W;
            J.start = total;
            J.area = (float)m.area;
            J.inv2dx = 0.5f * (float)m.W;
            J.inv2dy = 0.5f * (float)m.H;
            total += m.pdb;
            abc::RedJob& Rj = reds[j];
            std::memset(&Rj, 0, sizeof(Rj));
            Rj.part_f = m.pdpart;
            Rj.out_f = L.q_all + (size_t)j * abc::kPdQuantities;
            Rj.rows = 1;
            Rj.nblk = m.pdb;
        }
        ABC_HIP(hipMemcpyAsync(L.pix_jobs, jobs.data(), jobs.size() * sizeof(abc::PixJob), hipMemcpyHostToDevice, st));
        ABC_HIP(hipMemcpyAsync(L.red_jobs, reds.data(), reds.size() * sizeof(abc::RedJob), hipMemcpyHostToDevice, st));
        ABC_HIP(abc::launch_pd_step_batched(L.pix_jobs, (int)jobs.size(), total, update_mu, C, p->rho, p->gamma, st));
        if (!want) return ABC_OK;
        ABC_HIP(abc::launch_reduce_jobs(L.red_jobs, (int)reds.size(), abc::kPdQuantities, st));
        std::vector<float> q(who.size() * abc::kPdQuantities);
        ABC_HIP(hipMemcpyAsync(q.data(), L.q_all, q.size() * sizeof(float), hipMemcpyDeviceToHost, st));
        ABC_HIP(hipStreamSynchronize(st));
        for (size_t j = 0; j < who.size(); ++j) {
            Shape sh{im[who[j]].H, im[who[j]].W, C};
            energies_from(q.data() + j * abc::kPdQuantities, sh, p, &im[who[j]].E);
        }
        return ABC_OK;
    }

    void project(const BImg& m, double tau, std::vector<double>& out) const {
        for (int k = 0; k < K; ++k)
            for (int q = 0; q < 2; ++q) {
                const double x = m.e_base[2 * k + q] - tau * m.G[2 * k + q];
                out[2 * k + q] = std::min<double>(std::max<double>(x, p->eps_min[q]), p->eps_max[q]);
            }
    }
};

// abc_solve_batched tunes its tiles: asked for, with a window, and no tile given.
bool tunes_batch(const abc_params* p) {
    return (p->flags & ABC_FLAG_AUTOTUNE) && p->R > 0 && p->tile_x == 0 && p->tile_y == 0 && p->adj_tile_x == 0 &&
           p->adj_tile_y == 0;
}

// Tiles tuned by abc_solve_batched, kept for the process: keyed by GPU
// architecture, channels, radius and size class (the largest image's pixel
// count rounded up to a power of two).
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tuned;

size_t batch_ws_bytes(const int32_t* H, const int32_t* W, int n, int C, const abc_params* p, abc::Tile ta) {
    Carve cv(nullptr);
    BatchWs bw;
    carve_batch(cv, n, p->K, bw);
    for (int i = 0; i < n; ++i) {
        BImg m;
        m.H = H[i];
        m.W = W[i];
        m.f = (size_t)H[i] * W[i] * C;
        m.tiles_a = abc::tile_count(H[i], W[i], ta);
        m.pdb = abc::pd_blocks(H[i], W[i]);
        carve_bimg(cv, m, p->K, C);
    }
    return cv.used;
}

}  // namespace

extern "C" {

int abc_workspace_bytes_batched(const int32_t* H, const int32_t* W, int n, int C, const abc_params* p, size_t* bytes) {
    int rc = check_params(p);
    if (rc) return rc;
    if (p->R < 0 || p->R > ABC_MAX_RADIUS) return fail(ABC_EINVAL, "the batched solve takes R in [0, 16]");
    if (!H || !W || !bytes || n < 1) return fail(ABC_EINVAL, "H, W, bytes must be non-NULL and n >= 1");
    for (int i = 0; i < n; ++i)
        if ((rc = check_shape(H[i], W[i], C))) return rc;
    abc::Tile ta;
    if ((rc = pick_tile(p, C, 2, &ta))) return rc;
    *bytes = batch_ws_bytes(H, W, n, C, p, ta);
    if (tunes_batch(p)) {
        // the tuner may pick any admissible adjoint tile (the partials depend on it);
        // it runs in the workspace before the solve carves it
        int big = 0;
        for (int i = 1; i < n; ++i)
            if ((double)H[i] * W[i] > (double)H[big] * W[big]) big = i;
        *bytes = std::max(*bytes, tune_ws_bytes(H[big], W[big], C));
        for (const abc::Tile& t : kTuneCands)
            if (abc::tile_ok(C, p->R, t, 2)) *bytes = std::max(*bytes, batch_ws_bytes(H, W, n, C, p, t));
    }
    return ABC_OK;
}

int abc_solve_batched(const abc_image* imgs, int n, int C, const abc_params* p, void* ws, size_t ws_bytes,
                      void* stream, abc_stats* st, double* finish_ms, const abc_solve_log* logs) {
    Range range("abc_solve_batched");
    int rc = check_params(p);
    if (rc) return rc;
    if (p->R < 0 || p->R > ABC_MAX_RADIUS) return fail(ABC_EINVAL, "the batched solve takes R in [0, 16]");
    if (!imgs || n < 1) return fail(ABC_EINVAL, "imgs must be non-NULL and n >= 1");
    if (p->ckpt_every != 0) return fail(ABC_EINVAL, "abc_solve_batched stores full trajectories; set ckpt_every = 0");
    std::vector<int32_t> Hs(n), Ws(n);
    for (int i = 0; i < n; ++i) {
        if ((rc = check_shape(imgs[i].H, imgs[i].W, C))) return rc;
        if (!imgs[i].c0 || !imgs[i].c_out) return fail(ABC_EINVAL, "every image needs c0 and c_out");
        Hs[i] = imgs[i].H;
        Ws[i] = imgs[i].W;
        if (logs && logs[i].eps_replay && !logs[i].decisions_in)
            return fail(ABC_EINVAL, "eps_replay needs decisions_in");
    }
    abc_params pt = *p;  // p with the tuned tiles, when the tiles are tuned
    if (tunes_batch(p)) {
        int big = 0;
        for (int i = 1; i < n; ++i)
            if ((double)Hs[i] * Ws[i] > (double)Hs[big] * Ws[big]) big = i;
        int cls = 0;
        while (((int64_t)1 << cls) < (int64_t)Hs[big] * Ws[big]) ++cls;
        char keybuf[160];
        std::snprintf(keybuf, sizeof(keybuf), "%s|C=%d|R=%d|px<=2^%d", gpu_arch().c_str(), C, p->R, cls);
        TuneEntry te{0, 0, 0, 0, 0.0, 0.0};
        bool have = false;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tuned.find(keybuf);
            if (it != g_tuned.end()) {
                te = it->second;
                have = true;
            }
        }
        if (!have) {
            // the workspace is not in use yet: the tuner runs in it, on the largest image
            if (!ws || ws_bytes < tune_ws_bytes(Hs[big], Ws[big], C))
                return fail(ABC_EINVAL, "batched workspace too small for the tile tuner");
            if ((rc = tune_tiles(imgs[big].c0, Hs[big], Ws[big], C, p, ws, (hipStream_t)stream, &te))) return rc;
            std::lock_guard<std::mutex> lock(g_tune_mu);
            g_tuned[keybuf] = te;
        }
        pt.tile_x = te.ftx;
        pt.tile_y = te.fty;
        pt.adj_tile_x = te.atx;
        pt.adj_tile_y = te.aty;
    }
    p = &pt;
    Batch B;
    B.n = n;
    B.C = C;
    B.K = p->K;
    B.p = p;
    B.pq = *p;
    B.quad = p->cost == ABC_COST_QUADRATIC;
    if (B.quad) B.pq.rho = 1.0f;
    if ((rc = pick_tile(p, C, 1, &B.tf))) return rc;
    if ((rc = pick_tile(p, C, 2, &B.ta))) return rc;
    const size_t need = batch_ws_bytes(Hs.data(), Ws.data(), n, C, p, B.ta);
    if (!ws || ws_bytes < need) return fail(ABC_EINVAL, "batched workspace too small");
    B.st = (hipStream_t)stream;
    B.use_graphs = !(p->flags & ABC_FLAG_NO_GRAPHS) && p->R > 0;
    B.persistent = (p->flags & ABC_FLAG_PERSISTENT) != 0;
    const int K = p->K;
    Carve cv(ws);
    carve_batch(cv, n, K, B.w);
    B.w.a.st = B.st;
    ABC_HIP(hipStreamCreateWithFlags(&B.own_b, hipStreamNonBlocking));
    B.w.b.st = B.own_b;
    B.im.resize(n);
    B.eps_host.assign((size_t)n * 3 * K * 2, 0.0f);
    const auto t_start = std::chrono::steady_clock::now();
    auto now_ms = [&]() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    };
    for (int i = 0; i < n; ++i) {
        BImg& m = B.im[i];
        m.H = imgs[i].H;
        m.W = imgs[i].W;
        m.f = (size_t)m.H * m.W * C;
        m.tiles_f = abc::tile_count(m.H, m.W, B.tf);
        m.tiles_a = abc::tile_count(m.H, m.W, B.ta);
        m.pdb = abc::pd_blocks(m.H, m.W);
        Shape sh{m.H, m.W, C};
        m.snorm = norm_factor(p, sh);
        m.dts = p->dt * m.snorm;
        m.area = sh.area();
        carve_bimg(cv, m, K, C);
        m.c0 = imgs[i].c0;
        m.c_out = imgs[i].c_out;
        m.eps_user = imgs[i].eps;
        m.mu_user = imgs[i].mu;
        m.log = logs ? &logs[i] : nullptr;
        if (m.log) {
            const size_t nslots = (size_t)std::max(p->max_outer, 1) * std::max(p->max_inner, 1);
            if (m.log->decisions_out) std::fill(m.log->decisions_out, m.log->decisions_out + nslots, 0.0);
            if (m.log->grad_out) std::fill(m.log->grad_out, m.log->grad_out + nslots * 2 * K, 0.0);
            if (m.log->phi_out) std::fill(m.log->phi_out, m.log->phi_out + nslots * kStepLog, 0.0);
            if (m.log->outer_out) std::fill(m.log->outer_out, m.log->outer_out + (size_t)std::max(p->max_outer, 1) * 4, 0.0);
            if (m.log->eps_out) std::fill(m.log->eps_out, m.log->eps_out + nslots * 2 * K, 0.0);
        }
        m.e_base.assign((size_t)K * 2, (double)p->eps_init);
        m.e_try = m.e_cand = m.e_next = m.e_base;
        m.sigma = p->sigma0;
        std::memset(&m.S, 0, sizeof(m.S));
        std::memset(&m.E, 0, sizeof(m.E));
        m.S.gap_rel = NAN;
        m.S.K_start = NAN;
        m.S.ms_start = NAN;
        if (m.eps_user) {
            std::vector<float> h((size_t)K * 2);
            ABC_HIP(hipMemcpyAsync(h.data(), m.eps_user, h.size() * sizeof(float), hipMemcpyDeviceToHost, B.st));
            ABC_HIP(hipStreamSynchronize(B.st));
            for (int q = 0; q < 2 * K; ++q) {
                if (!std::isfinite(h[q])) return fail(ABC_ENONFINITE, "controls hold a NaN or Inf");
                m.e_base[q] = h[q];
            }
        }
        // slot 0 of every trajectory buffer holds c0 for the whole solve
        for (int b = 0; b < 3; ++b)
            ABC_HIP(hipMemcpyAsync(m.traj[b], m.c0, m.f * sizeof(float), hipMemcpyDeviceToDevice, B.st));
        if (m.mu_user && !B.quad)
            ABC_HIP(hipMemcpyAsync(m.mu, m.mu_user, 2 * m.f * sizeof(float), hipMemcpyDeviceToDevice, B.st));
        else
            ABC_HIP(hipMemsetAsync(m.mu, 0, 2 * m.f * sizeof(float), B.st));
        if (B.quad) ABC_HIP(hipMemsetAsync(m.v, 0, 2 * m.f * sizeof(float), B.st));
    }
    std::vector<int> all(n), slots;
    for (int i = 0; i < n; ++i) all[i] = i;
    {
        std::vector<int> s0(n, 0);
        std::vector<const std::vector<double>*> vals(n);
        for (int i = 0; i < n; ++i) vals[i] = &B.im[i].e_base;
        if ((rc = B.upload_eps(all, s0, vals, B.st))) return rc;
        if ((rc = B.forward(all, s0, B.w.a))) return rc;
        if (!B.quad && (rc = B.pd(all, 0, false))) return rc;
    }
    const int M = B.quad ? std::min(p->max_outer, 1) : p->max_outer;
    const int P = p->max_inner;
    std::vector<double> phi;
    // Each image runs its own loops (Alg. 2 around Alg. 1).  A round gives
    // every image one step of its own: a gradient, one Armijo trial, or a
    // multiplier update; the images in each phase share one launch per Euler
    // step, and the trial sweeps run on a second stream while the gradient
    // sweeps run on the caller's.  Images never wait for each other at a
    // multiplier iteration, so a small image finishes early.  Every use of an
    // image's buffers on one stream follows a host wait on the other.
    auto end_inner = [&](BImg& m) { m.phase = kPhPd; };
    for (int i = 0; i < n; ++i) B.im[i].phase = M > 0 ? kPhGrad : kPhDone;
    for (int i = 0; i < n; ++i)
        if (M > 0 && P == 0) end_inner(B.im[i]);
    auto in_phase = [&](int ph) {
        std::vector<int> v;
        for (int i = 0; i < n; ++i)
            if (B.im[i].phase == ph) v.push_back(i);
        return v;
    };
    std::vector<double> phi_s, K_s;
    for (;;) {
        Range round_range("batched round");
        std::vector<int> act = in_phase(kPhGrad);
        std::vector<int> search = in_phase(kPhSearch);
        std::vector<int> pdset = in_phase(kPhPd);
        if (act.empty() && search.empty() && pdset.empty()) break;
        // queue one Armijo trial for every image in a search (lane b)
        if (!search.empty()) {
            std::vector<int> tslot;
            std::vector<const std::vector<double>*> vals;
            for (int i : search) {
                BImg& m = B.im[i];
                const size_t slot = (size_t)m.j * P + (m.it - 1);
                if (m.log && m.log->eps_replay)
                    m.e_try.assign(m.log->eps_replay + slot * 2 * K, m.log->eps_replay + (slot + 1) * 2 * K);
                else
                    B.project(m, m.tau, m.e_try);
                tslot.push_back(m.trial);
                vals.push_back(&m.e_try);
            }
            if ((rc = B.upload_eps(search, tslot, vals, B.w.b.st))) return rc;
            if ((rc = B.forward(search, tslot, B.w.b))) return rc;
            if ((rc = B.objective_launch(search, tslot, false, B.w.b))) return rc;
        }
        // gradients (lane a)
        if (!act.empty()) {
            std::vector<int> bslot;
            for (int i : act) bslot.push_back(B.im[i].base);
            if ((rc = B.objective(act, bslot, true, phi, B.w.a))) return rc;
            if ((rc = B.adjoint(act))) return rc;
            for (size_t a = 0; a < act.size(); ++a) {
                BImg& m = B.im[act[a]];
                m.phi0 = phi[a];
                if (!m.phi_seen) {
                    m.S.phi_first = m.phi0;
                    m.phi_seen = true;
                }
                m.S.phi_last = m.phi0;
                m.S.inner_iters++;
                m.it++;
                const size_t slot = (size_t)m.j * P + (m.it - 1);
                const abc_solve_log* lg = m.log;
                if (lg && lg->grad_out) std::copy(m.G.begin(), m.G.end(), lg->grad_out + slot * 2 * K);
                if (lg && lg->phi_out) lg->phi_out[kStepLog * slot] = m.phi0;
                bool all_zero = true;
                for (double g : m.G) all_zero = all_zero && (g == 0.0);
                const bool replay = lg && lg->decisions_in;
                if (replay ? !(lg->decisions_in[slot] > 0.0) : all_zero) {
                    end_inner(m);
                    continue;
                }
                m.tau = replay ? lg->decisions_in[slot] : m.sigma;
                m.evals = 0;
                m.branch = 0;
                m.have = false;
                m.ls_done = false;
                m.accepted = 0.0;
                m.phi_acc = m.phi0;
                m.phase = kPhSearch;
            }
        }
        // Armijo decisions of the trials
        if (!search.empty()) {
            if ((rc = B.objective_read(search, B.w.b, phi_s, &K_s))) return rc;
            for (size_t a = 0; a < search.size(); ++a) {
                BImg& m = B.im[search[a]];
                const size_t slot = (size_t)m.j * P + (m.it - 1);
                const abc_solve_log* lg = m.log;
                const bool replay = lg && lg->decisions_in;
                m.evals++;
                double ip = 0.0;
                for (int q = 0; q < 2 * K; ++q) ip += m.G[q] * (m.e_try[q] - m.e_base[q]);
                ip *= (double)p->dt;
                const bool ok = phi_s[a] <= m.phi0 + p->armijo_c * ip;
                auto keep = [&]() {
                    std::swap(m.cand, m.trial);
                    m.e_cand = m.e_try;
                    m.accepted = m.tau;
                    m.phi_acc = phi_s[a];
                    m.K_acc = K_s[a];
                    m.have = true;
                };
                bool more = false;
                if (replay) {
                    // a replayed step is taken as recorded; with replayed controls the
                    // step this iteration's own gradient gives is logged
                    if (lg->eps_replay && lg->eps_out) {
                        B.project(m, m.tau, m.e_next);
                        std::copy(m.e_next.begin(), m.e_next.end(), lg->eps_out + slot * 2 * K);
                    }
                    keep();
                    m.ls_done = true;
                } else if (m.branch == 0) {
                    if (ok) {
                        keep();
                        m.branch = 1;
                    } else {
                        m.branch = 2;
                    }
                } else if (m.branch == 1) {
                    if (ok) keep();
                    else m.ls_done = true;
                } else {
                    if (ok) {
                        keep();
                        m.ls_done = true;
                    }
                }
                if (!m.ls_done && m.evals < p->max_ls) {
                    if (m.branch == 1) {
                        B.project(m, m.tau / p->armijo_b, m.e_next);
                        if (m.e_next != m.e_cand) {
                            m.tau /= p->armijo_b;
                            more = true;
                        }
                    } else {
                        m.tau *= p->armijo_b;
                        more = true;
                    }
                }
                if (more) continue;
                m.S.ls_evals += m.evals;
                if (lg && lg->phi_out) lg->phi_out[kStepLog * slot + 2] = m.evals;
                if (!m.have) {
                    end_inner(m);
                    continue;
                }
                if (!replay) m.sigma = m.accepted;
                m.e_base = m.e_cand;
                std::swap(m.base, m.cand);
                if (lg) {
                    if (lg->decisions_out) lg->decisions_out[slot] = m.accepted;
                    if (lg->eps_out && !lg->eps_replay)
                        std::copy(m.e_base.begin(), m.e_base.end(), lg->eps_out + slot * 2 * K);
                    if (lg->phi_out) {
                        lg->phi_out[kStepLog * slot + 1] = m.phi_acc;
                        lg->phi_out[kStepLog * slot + 3] = m.K_acc;
                        lg->phi_out[kStepLog * slot + 4] = now_ms();
                    }
                }
                if ((p->tol_dal > 0.0 && std::fabs(m.phi_acc - m.phi0) < p->tol_dal * std::fabs(m.phi0)) ||
                    m.it >= P)
                    end_inner(m);
                else
                    m.phase = kPhGrad;
            }
        }
        // multiplier updates
        pdset = in_phase(kPhPd);
        if (pdset.empty()) continue;
        if (B.quad) {
            for (int i : pdset) {
                B.im[i].S.outer_iters = 1;
                B.im[i].outer_done = true;
                B.im[i].phase = kPhDone;
                B.im[i].finish_ms = now_ms();
            }
            continue;
        }
        if ((rc = B.pd(pdset, 1, true))) return rc;
        const double t_now = now_ms();
        for (int i : pdset) {
            BImg& m = B.im[i];
            m.S.outer_iters = m.j + 1;
            m.S.gap_rel = std::isnan(m.L_prev) ? NAN : std::fabs(m.E.L - m.L_prev) / std::fabs(m.L_prev);
            m.L_prev = m.E.L;
            if (m.log && m.log->outer_out) {
                double* o = m.log->outer_out + 4 * (size_t)m.j;
                o[0] = m.E.K;
                o[1] = m.E.L;
                o[2] = m.E.r_rel;
                o[3] = t_now;
            }
            const bool gap_ok = p->tol_gap > 0.0 && !std::isnan(m.S.gap_rel) && m.S.gap_rel < p->tol_gap;
            if ((p->tol_alm > 0.0 && m.E.r_rel < p->tol_alm) || (p->stop_K > 0.0 && m.E.K <= p->stop_K) || gap_ok ||
                m.j + 1 == M) {
                m.outer_done = true;
                m.phase = kPhDone;
                m.finish_ms = t_now;
            } else {
                m.j++;
                m.it = 0;
                m.phase = P > 0 ? kPhGrad : kPhPd;
            }
        }
    }
    // outputs
    int status = ABC_OK;
    std::vector<int> final_e;
    for (int i = 0; i < n; ++i) {
        BImg& m = B.im[i];
        if (!m.outer_done) m.finish_ms = now_ms();
        ABC_HIP(hipMemcpyAsync(m.c_out, m.traj[m.base] + (size_t)K * m.f, m.f * sizeof(float),
                               hipMemcpyDeviceToDevice, B.st));
        if (m.eps_user) {
            std::vector<float> h((size_t)K * 2);
            for (int q = 0; q < 2 * K; ++q) h[q] = (float)m.e_base[q];
            ABC_HIP(hipMemcpyAsync(m.eps_user, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, B.st));
            ABC_HIP(hipStreamSynchronize(B.st));
        }
        if (m.mu_user && !B.quad)
            ABC_HIP(hipMemcpyAsync(m.mu_user, m.mu, 2 * m.f * sizeof(float), hipMemcpyDeviceToDevice, B.st));
        if (B.quad || m.S.outer_iters == 0) final_e.push_back(i);
    }
    if (!final_e.empty()) {
        // energies where no multiplier update ran: the pd kernel on zeroed scratch (spare trajectories)
        for (int i : final_e) {
            BImg& m = B.im[i];
            float* sv = m.traj[m.trial];
            float* sm = m.traj[m.cand];
            if (B.quad || m.S.outer_iters == 0) {
                ABC_HIP(hipMemsetAsync(sv, 0, 2 * m.f * sizeof(float), B.st));
                ABC_HIP(hipMemcpyAsync(sm, m.mu, 2 * m.f * sizeof(float), hipMemcpyDeviceToDevice, B.st));
                if (B.quad) ABC_HIP(hipMemsetAsync(sm, 0, 2 * m.f * sizeof(float), B.st));
                std::swap(m.v, sv);
                std::swap(m.mu, sm);
            }
        }
        if ((rc = B.pd(final_e, 0, true))) return rc;
        if (B.quad) {
            std::vector<int> bslot;
            for (int i : final_e) bslot.push_back(B.im[i].base);
            // the quadratic objective is evaluated with v = mu = 0
            for (int i : final_e) {
                BImg& m = B.im[i];
                ABC_HIP(hipMemsetAsync(m.v, 0, 2 * m.f * sizeof(float), B.st));
                ABC_HIP(hipMemsetAsync(m.mu, 0, 2 * m.f * sizeof(float), B.st));
            }
            if ((rc = B.objective(final_e, bslot, false, phi, B.w.a))) return rc;
            for (size_t a = 0; a < final_e.size(); ++a) {
                BImg& m = B.im[final_e[a]];
                m.E.L = m.E.Ltilde = phi[a];
                m.E.r_rel = m.E.r_abs = 0.0;
            }
        }
    }
    ABC_HIP(hipStreamSynchronize(B.st));
    for (int i = 0; i < n; ++i) {
        BImg& m = B.im[i];
        abc_stats S = m.S;
        S.K = m.E.K;
        S.TV = m.E.TV;
        S.fid = m.E.fid;
        S.L = m.E.L;
        S.Ltilde = m.E.Ltilde;
        S.r_rel = m.E.r_rel;
        S.r_abs = m.E.r_abs;
        S.status = (!B.quad && p->tol_alm > 0.0 && !(m.E.r_rel < p->tol_alm)) ? ABC_ENOCONV : ABC_OK;
        if (S.status) status = ABC_ENOCONV;
        if (st) st[i] = S;
        if (finish_ms) finish_ms[i] = m.finish_ms;
    }
    return status;
}

}  // extern "C"

// ===========================================================================
// Tile autotuner with a JSON cache.
extern "C" int abc_autotune(const float* c0, int H, int W, int C, abc_params* p, const char* cache_path, void* ws,
                            size_t ws_bytes, void* stream, double* best_us) {
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_shape(H, W, C))) return rc;
    if (p->R == ABC_RADIUS_SUPPORT) {
        // tune for the resolved radius; p keeps asking for the support radius
        abc_params pr;
        pr = *with_radius(p, H, W, pr);
        if ((rc = abc_autotune(c0, H, W, C, &pr, cache_path, ws, ws_bytes, stream, best_us))) return rc;
        p->tile_x = pr.tile_x;
        p->tile_y = pr.tile_y;
        p->adj_tile_x = pr.adj_tile_x;
        p->adj_tile_y = pr.adj_tile_y;
        return ABC_OK;
    }
    if (!c0) return fail(ABC_EINVAL, "c0 must be non-NULL");
    if (best_us) best_us[0] = best_us[1] = 0.0;
    if (p->R == 0) return ABC_OK;
    char keybuf[160];
    std::snprintf(keybuf, sizeof(keybuf), "%s|C=%d|R=%d|H=%d|W=%d", gpu_arch().c_str(), C, p->R, H, W);
    const std::string key(keybuf);
    std::map<std::string, TuneEntry> cache = read_tune_cache(cache_path);
    auto hit = cache.find(key);
    if (hit != cache.end() && abc::tile_ok(C, p->R, abc::Tile{hit->second.ftx, hit->second.fty}, 1) &&
        abc::tile_ok(C, p->R, abc::Tile{hit->second.atx, hit->second.aty}, 2)) {
        p->tile_x = hit->second.ftx;
        p->tile_y = hit->second.fty;
        p->adj_tile_x = hit->second.atx;
        p->adj_tile_y = hit->second.aty;
        return ABC_OK;
    }
    if (!ws || ws_bytes < tune_ws_bytes(H, W, C)) return fail(ABC_EINVAL, "autotune workspace too small");
    TuneEntry best;
    if ((rc = tune_tiles(c0, H, W, C, p, ws, (hipStream_t)stream, &best))) return rc;
    p->tile_x = best.ftx;
    p->tile_y = best.fty;
    p->adj_tile_x = best.atx;
    p->adj_tile_y = best.aty;
    if (best_us) {
        best_us[0] = best.fus;
        best_us[1] = best.aus;
    }
    if (cache_path) {
        cache[key] = best;
        if (!write_tune_cache(cache_path, cache)) return fail(ABC_EINVAL, std::string("cannot write ") + cache_path);
    }
    return ABC_OK;
}

namespace abc {
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace abc
