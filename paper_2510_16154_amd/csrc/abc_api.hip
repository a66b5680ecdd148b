// Host side of the C ABI declared in include/abc.h: argument checks, workspace
// carving, the forward and adjoint sweeps, and the solver loop (method of
// multipliers, Alg. 2, with the direct-adjoint / two-way Armijo control argmin
// of Alg. 1).  Decisions of the line search are taken in FP64 on the host from
// FP32 device reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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
    if ((double)H * (double)W * (double)C > 4.0e9) return fail(ABC_EINVAL, "image too large");
    return ABC_OK;
}

int check_params(const abc_params* p) {
    if (!p) return fail(ABC_EINVAL, "params is NULL");
    if (p->K < 1) return fail(ABC_EINVAL, "K must be >= 1");
    if (p->R < 0 || p->R > ABC_MAX_RADIUS) return fail(ABC_EINVAL, "R must be in [0, 16]");
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
    return ABC_OK;
}

int pick_tile(const abc_params* p, int C, int fields, abc::Tile* t) {
    if (p->tile_x > 0 || p->tile_y > 0) {
        abc::Tile u{p->tile_x, p->tile_y};
        if (!abc::tile_ok(C, p->R, u, fields))
            return fail(ABC_EINVAL, "tile_x * tile_y must be a multiple of 64 and <= 256, and fit in LDS");
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
        case ABC_WS_SOLVE: carve_solve(cv, s, p, abc::tile_count(s.H, s.W, ta)); break;
        case ABC_WS_FORWARD:
            if (p->ckpt_every > 0) cv.take<float>(2 * s.field());
            break;
        case ABC_WS_ADJOINT: carve_adjoint(cv, s, p, abc::tile_count(s.H, s.W, ta)); break;
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

// Reduced control gradient: G[k][m] (FP64) = dl/deps^k_m / dt = -5 s * (raw sums).
int fetch_gradient(const double* part, int K, int tiles, double* Gdev, float s_norm, hipStream_t st,
                   std::vector<double>& G) {
    ABC_HIP(abc::launch_reduce_rows_f64(part, K, tiles, 2, -5.0 * (double)s_norm, Gdev, nullptr, st));
    G.resize((size_t)K * 2);
    ABC_HIP(hipMemcpyAsync(G.data(), Gdev, G.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    ABC_HIP(hipStreamSynchronize(st));
    return ABC_OK;
}

int objective(const float* cK, const float* c0, const float* v, const float* mu, float* pK, const Shape& s,
              const abc_params* p, const PdWs& w, hipStream_t st, double* phi) {
    ABC_HIP(abc::launch_terminal(cK, c0, v, mu, s.H, s.W, s.C, p->rho, p->alpha, (float)s.area(), pK, w.part, st));
    if (!phi) return ABC_OK;
    ABC_HIP(abc::launch_reduce_rows(w.part, 1, abc::pd_blocks(s.H, s.W), 1, w.out, 1.0f, st));
    float h = 0.0f;
    ABC_HIP(hipMemcpyAsync(&h, w.out, sizeof(float), hipMemcpyDeviceToHost, st));
    ABC_HIP(hipStreamSynchronize(st));
    *phi = s.area() * (double)h;
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
    float q[abc::kPdQuantities];
    ABC_HIP(hipMemcpyAsync(q, w.out, sizeof(q), hipMemcpyDeviceToHost, st));
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

// ===========================================================================
extern "C" {

int abc_version(void) { return 100; }

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
    if (!bytes) return fail(ABC_EINVAL, "bytes is NULL");
    if (kind < ABC_WS_SOLVE || kind > ABC_WS_PD) return fail(ABC_EINVAL, "unknown workspace kind");
    abc::Tile tf{32, 8}, ta{32, 8};
    if ((rc = pick_tile(p, C, 1, &tf))) return rc;
    if ((rc = pick_tile(p, C, 2, &ta))) return rc;
    *bytes = ws_bytes_for(kind, Shape{H, W, C}, p, tf, ta);
    return ABC_OK;
}

int abc_forward_dynamics(const float* c0, int H, int W, int C, const float* eps, const abc_params* p, float* traj,
                         void* ws, size_t ws_bytes, void* stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_shape(H, W, C))) return rc;
    if (!c0 || !eps || !traj) return fail(ABC_EINVAL, "c0, eps and traj must be non-NULL");
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
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_shape(H, W, C))) return rc;
    if (!traj || !eps || !gK || !g0 || !geps) return fail(ABC_EINVAL, "traj, eps, gK, g0, geps must be non-NULL");
    const Shape s{H, W, C};
    abc::Tile tf, ta;
    if ((rc = pick_tile(p, C, 1, &tf))) return rc;
    if ((rc = pick_tile(p, C, 2, &ta))) return rc;
    const size_t need = ws_bytes_for(ABC_WS_ADJOINT, s, p, tf, ta);
    if (!ws || ws_bytes < need) return fail(ABC_EINVAL, "adjoint workspace too small");
    hipStream_t st = (hipStream_t)stream;
    const size_t f = s.field();
    const int tiles = abc::tile_count(H, W, ta);
    Carve cv(ws);
    AdjointWs w = carve_adjoint(cv, s, p, tiles);
    const float snorm = norm_factor(p, s);
    const float dts = p->dt * snorm;
    if (p->R == 0) {
        if (g0 != gK) ABC_HIP(hipMemcpyAsync(g0, gK, f * sizeof(float), hipMemcpyDeviceToDevice, st));
        ABC_HIP(hipMemsetAsync(geps, 0, (size_t)p->K * 2 * sizeof(float), st));
        return ABC_OK;
    }
    ABC_HIP(hipMemcpyAsync(w.pa, gK, f * sizeof(float), hipMemcpyDeviceToDevice, st));
    float* cur = w.pa;
    float* spare = w.pb;
    if (p->ckpt_every <= 0) {
        std::vector<const float*> states(p->K);
        for (int k = 0; k < p->K; ++k) states[k] = traj + (size_t)k * f;
        if ((rc = adjoint_steps(states.data(), 0, p->K, eps, s, p, dts, ta, cur, spare, w.part, tiles, st)))
            return rc;
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
            if ((rc = adjoint_steps(states.data(), k0, k1, eps, s, p, dts, ta, cur, spare, w.part, tiles, st)))
                return rc;
        }
    }
    ABC_HIP(hipMemcpyAsync(g0, cur, f * sizeof(float), hipMemcpyDeviceToDevice, st));
    // dl/deps^k = -5 dt s * (raw sums of the adjoint kernel), summed in FP64
    ABC_HIP(abc::launch_reduce_rows_f64(w.part, p->K, tiles, 2, -5.0 * (double)p->dt * (double)snorm, nullptr, geps,
                                        st));
    return ABC_OK;
}

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
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_shape(H, W, C))) return rc;
    if (!c0 || !c_out) return fail(ABC_EINVAL, "c0 and c_out must be non-NULL");
    if (p->ckpt_every != 0) return fail(ABC_EINVAL, "abc_solve stores full trajectories; set ckpt_every = 0");
    const double* decisions_in = log ? log->decisions_in : nullptr;
    double* decisions_out = log ? log->decisions_out : nullptr;
    const double* eps_replay = log ? log->eps_replay : nullptr;
    double* grad_out = log ? log->grad_out : nullptr;
    double* phi_out = log ? log->phi_out : nullptr;
    if (eps_replay && !decisions_in) return fail(ABC_EINVAL, "eps_replay needs decisions_in");
    const Shape s{H, W, C};
    abc::Tile tf, ta;
    if ((rc = pick_tile(p, C, 1, &tf))) return rc;
    if ((rc = pick_tile(p, C, 2, &ta))) return rc;
    const size_t need = ws_bytes_for(ABC_WS_SOLVE, s, p, tf, ta);
    if (!ws || ws_bytes < need) return fail(ABC_EINVAL, "solve workspace too small");
    hipStream_t st = (hipStream_t)stream;
    const int K = p->K;
    const size_t f = s.field();
    const int tiles = abc::tile_count(H, W, ta);
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

    auto upload = [&](const std::vector<double>& e, float* dev) -> int {
        std::vector<float> h(e.size());
        for (size_t i = 0; i < e.size(); ++i) h[i] = (float)e[i];
        ABC_HIP(hipMemcpyAsync(dev, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, st));
        ABC_HIP(hipStreamSynchronize(st));
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
    // Armijo trial into buffer `trial`: eps(tau), forward sweep, Phi(tau), test.
    auto run_trial = [&](const std::vector<double>& G, double tau, double phi0, double* phit, bool* ok) -> int {
        project(G, tau, e_try);
        int r2 = upload(e_try, w.eps[trial]);
        if (r2) return r2;
        if ((r2 = forward_sweep_full(c0, w.traj[trial], w.eps[trial], s, p, dts, tf, st))) return r2;
        if ((r2 = objective(w.traj[trial] + traj_stride, c0, vv, mm, nullptr, s, &pq, w.pd, st, phit))) return r2;
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
    if (phi_out) std::fill(phi_out, phi_out + nslots * 3, 0.0);

    // Alg. 2: forward integration, v^(0) = argmin_v L(c^(0), v, mu^(0)).
    if ((rc = upload(e_base, w.eps[base]))) return rc;
    if ((rc = forward_sweep_full(c0, w.traj[base], w.eps[base], s, p, dts, tf, st))) return rc;
    if (!quad && (rc = pd_update(w.traj[base] + traj_stride, c0, vv, mm, 0, s, p, w.pd, st, nullptr))) return rc;

    double sigma = p->sigma0;
    double L_prev = NAN;
    bool phi_seen = false;
    abc_stats E;
    std::memset(&E, 0, sizeof(E));
    std::vector<double> G;
    const int n_outer = quad ? std::min(M, 1) : M;
    for (int j = 0; j < n_outer; ++j) {
        for (int it = 0; it < P; ++it) {
            const size_t slot = (size_t)j * P + it;
            double phi0 = 0.0;
            if ((rc = objective(w.traj[base] + traj_stride, c0, vv, mm, w.adj.pa, s, &pq, w.pd, st, &phi0))) return rc;
            if (!phi_seen) {
                S.phi_first = phi0;
                phi_seen = true;
            }
            S.phi_last = phi0;
            // adjoint sweep from p^K = dL~/dc, then the control gradient
            float* cur = w.adj.pa;
            float* spare = w.adj.pb;
            if (p->R > 0) {
                std::vector<const float*> states(K);
                for (int k = 0; k < K; ++k) states[k] = w.traj[base] + (size_t)k * f;
                if ((rc = adjoint_steps(states.data(), 0, K, w.eps[base], s, p, dts, ta, cur, spare, w.adj.part,
                                        tiles, st)))
                    return rc;
                if ((rc = fetch_gradient(w.adj.part, K, tiles, w.G, snorm, st, G))) return rc;
            } else {
                G.assign((size_t)K * 2, 0.0);
            }
            S.inner_iters++;
            if (grad_out) std::copy(G.begin(), G.end(), grad_out + slot * 2 * K);
            if (phi_out) phi_out[3 * slot] = phi0;
            bool all_zero = true;
            for (double g : G) all_zero = all_zero && (g == 0.0);
            if (decisions_in && !(decisions_in[slot] > 0.0)) break;
            if (!decisions_in && all_zero) break;

            double accepted = 0.0, phi_acc = phi0;
            if (decisions_in) {
                accepted = decisions_in[slot];
                bool ok = false;
                if (eps_replay) {
                    e_try.assign(eps_replay + slot * 2 * K, eps_replay + (slot + 1) * 2 * K);
                    if ((rc = upload(e_try, w.eps[trial]))) return rc;
                    if ((rc = forward_sweep_full(c0, w.traj[trial], w.eps[trial], s, p, dts, tf, st))) return rc;
                    if ((rc = objective(w.traj[trial] + traj_stride, c0, vv, mm, nullptr, s, &pq, w.pd, st, &phi_acc)))
                        return rc;
                } else if ((rc = run_trial(G, accepted, phi0, &phi_acc, &ok))) {
                    return rc;
                }
                std::swap(cand, trial);
                e_cand = e_try;
                S.ls_evals++;
                if (phi_out) phi_out[3 * slot + 2] = 1;
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
                            have = true;
                            break;
                        }
                    }
                }
                S.ls_evals += evals;
                if (phi_out) phi_out[3 * slot + 2] = evals;
                if (!have) break;
                sigma = accepted;
            }
            e_base = e_cand;
            std::swap(base, cand);
            if (decisions_out) decisions_out[slot] = accepted;
            if (phi_out) phi_out[3 * slot + 1] = phi_acc;
            if (p->tol_dal > 0.0 && std::fabs(phi_acc - phi0) < p->tol_dal * std::fabs(phi0)) break;
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
        if (p->tol_alm > 0.0 && E.r_rel < p->tol_alm) break;
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
    } else if (S.outer_iters == 0) {
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
    if (stats) *stats = S;
    return S.status;
}

}  // extern "C"
