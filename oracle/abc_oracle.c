/*
 * FP64 CPU oracle for the agent-based optimal-control solver of
 * "Agent-Based Optimal Control for Image Processing" (Oliviero, Cacace,
 * Visconti, arXiv 2510.16154).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library and must never be used as a
 * fallback for it.
 *
 * Everything is plain double precision, straight loops, no fast-math, no
 * blocking or fusion beyond what the definitions below state.  The only
 * parallelism is an OpenMP loop over image rows; every reduction goes into
 * per-row partial sums that are then added serially in row order, so results
 * do not depend on the thread count.
 *
 * Data layout (chosen for this project, the paper stores grey images as an
 * N_R x N_C matrix, Sec. 2):
 *   colour fields  c[(r*W + q)*C + ch]          (H x W x C, channel fastest)
 *   2-vector fields w[((r*W + q)*2 + d)*C + ch]  d = 0: along columns (x),
 *                                                d = 1: along rows (y)
 *   controls       eps[k*2 + 0] = eps_x^k, eps[k*2 + 1] = eps_c^k
 * Row index r runs along y; the paper orders rows bottom to top (Sec. 2),
 * which only flips the sign of y-components of v and mu.
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *  - Kernel: Wendland's C^2 function (1+4r)(1-r)^4 on [0,1]; the printed
 *    (4r-1)(1-r)^4 (Sec. 3.2, eq. kernel) gives phi(0) = -1 and is read as a
 *    sign typo.  The literal form is available through or_phi_literal().
 *  - Positions are normalised (dx = 1/W, dy = 1/H, Def. 3.1); the
 *    interaction sum runs over a square window of radius R clipped at the
 *    image border and is scaled by s (1/N in eq. MAsystem; the caller
 *    chooses s).
 *  - Explicit Euler with piecewise-constant controls (eps^k on step k).
 *  - Adjoint: the exact discrete transpose of the Euler step ("gradient
 *    sign": p = dl/dc, i.e. p = -lambda of eq. opt_system).
 *  - div := -(grad#)^T, so the terminal condition of eq. admm_terminal is
 *    the exact gradient of the completed-square functional (eq.
 *    complete_square); it equals the printed div# away from the border.
 *  - Armijo: two-way search on the projected path eps(tau) = Pi_E(eps - tau
 *    G) with the projected sufficient-decrease test, sigma set to the last
 *    step that passed (Alg. 1 with its sign typo in the update read as
 *    eps - sigma G).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-4)

/* ------------------------------------------------------------------ */
/* Parameters of the solver (own definition, independent of the GPU ABI) */
typedef struct {
    int K;             /* number of explicit Euler steps                  */
    double dt;         /* time step (Sec. 3.2: 0.25)                      */
    int R;             /* interaction window radius in pixels             */
    double s;          /* normalisation of the interaction sum (1/N)      */
    double eps_min[2]; /* control box E (Sec. 3.2: [2,1100]^2)            */
    double eps_max[2];
    double eps_init;   /* initial control (Sec. 3.2: 57)                  */
    double alpha;      /* fidelity weight                                 */
    double rho;        /* penalty parameter (Sec. 4.2: 1e-2)              */
    double gamma;      /* dual ascent step (Sec. 4.2: 1e-2)               */
    int max_outer;     /* multiplier iterations M                         */
    int max_inner;     /* DAL iterations per control argmin P             */
    int max_ls;        /* cap on Armijo trials per DAL iteration          */
    double tol_alm;    /* stop when r_rel < tol_alm (0: run M)            */
    double tol_dal;    /* relative stationarity of the inner cost         */
    double sigma0;     /* initial Armijo step (Sec. 3.2: 1)               */
    double armijo_b;   /* step factor (Sec. 3.2: 1/2)                     */
    double armijo_c;   /* sufficient decrease (Sec. 3.2: 1e-4)            */
    int literal_kernel;/* 1: use the printed (4r-1)(1-r)^4 (debug only)   */
    int cost;          /* 0: TV cost, method of multipliers (Alg. 2);
                          1: quadratic cost J (Def. 3.2), DAL alone (Alg. 1) */
    double tol_gap;    /* stop when |L_j - L_{j-1}| / |L_{j-1}| < tol_gap (0: off) */
} or_params;

/* Results of one primal/dual update or energy evaluation. */
typedef struct {
    double TV, fid, K, L, Ltilde;   /* energies (eq. cost_TV, eq. cost_tv_regular, eq. complete_square) */
    double r_abs, r_rel;            /* residual of v - grad c                    */
    double sq_vg, sq_g, sq_v;       /* raw sums of squares behind r_rel          */
} or_energies;

/* Statistics of a full solve. */
typedef struct {
    int status;        /* 0 converged / ran to caps, 1 caps hit before tol_alm */
    int outer_iters, inner_iters, ls_evals;
    double K, TV, fid, L, Ltilde, r_rel, r_abs, gap_rel;
    double phi_first, phi_last; /* inner objective at the first and last DAL step */
} or_stats;

/* ------------------------------------------------------------------ */
/* Interaction kernel (Sec. 3.2, eq. kernel; Wendland C^2 function).   */
double or_phi(double r)
{
    if (r < 0.0 || r > 1.0) return 0.0;
    double t = 1.0 - r;
    return (1.0 + 4.0 * r) * t * t * t * t;
}

/* d phi / dr = -20 r (1-r)^3 on [0,1]. */
double or_dphi(double r)
{
    if (r < 0.0 || r > 1.0) return 0.0;
    double t = 1.0 - r;
    return -20.0 * r * t * t * t;
}

/* The kernel exactly as printed, kept only to show what the sign reading changes. */
double or_phi_literal(double r)
{
    if (r < 0.0 || r > 1.0) return 0.0;
    double t = 1.0 - r;
    return (4.0 * r - 1.0) * t * t * t * t;
}

double or_dphi_literal(double r)
{
    if (r < 0.0 || r > 1.0) return 0.0;
    double t = 1.0 - r;
    /* d/dr[(4r-1) t^4] = 4 t^4 - 4 (4r-1) t^3 = t^3 (8 - 20 r) */
    return t * t * t * (8.0 - 20.0 * r);
}

static double kern(const or_params* P, double r)
{
    return P->literal_kernel ? or_phi_literal(r) : or_phi(r);
}

static double dkern(const or_params* P, double r)
{
    return P->literal_kernel ? or_dphi_literal(r) : or_dphi(r);
}

/* ------------------------------------------------------------------ */
/* Forward dynamics (eq. MAsystem with the distance of eq. ellipsoid),  */
/* one explicit Euler step:                                             */
/*   c_i <- c_i + dt * s * sum_{j in W(i)} phi(r_ij) (c_j - c_i),       */
/*   r_ij = ex/2 |x_j - x_i|^2 + ec/2 |c_j - c_i|^2.                    */
int or_forward_step(const double* c, double* cn, int H, int W, int C,
                    const or_params* P, double ex, double ec)
{
    const double dx = 1.0 / W, dy = 1.0 / H;
    const int R = P->R;
    /* per-row scratch: the force F and the differences d of one pixel */
    double* scratch = (double*)malloc(sizeof(double) * 2 * (size_t)H * (size_t)C);
    if (!scratch) return OR_ENOMEM;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < H; ++r) {
        double* F = scratch + 2 * (size_t)r * C;
        double* d = F + C;
        for (int q = 0; q < W; ++q) {
            const double* ci = c + ((size_t)r * W + q) * C;
            for (int ch = 0; ch < C; ++ch) F[ch] = 0.0;
            for (int a = -R; a <= R; ++a) {
                int rr = r + a;
                if (rr < 0 || rr >= H) continue;
                for (int b = -R; b <= R; ++b) {
                    int qq = q + b;
                    if (qq < 0 || qq >= W) continue;
                    const double* cj = c + ((size_t)rr * W + qq) * C;
                    double d2 = (b * dx) * (b * dx) + (a * dy) * (a * dy);
                    double n2 = 0.0;
                    for (int ch = 0; ch < C; ++ch) {
                        d[ch] = cj[ch] - ci[ch];
                        n2 += d[ch] * d[ch];
                    }
                    double rij = 0.5 * ex * d2 + 0.5 * ec * n2;
                    double w = kern(P, rij);
                    for (int ch = 0; ch < C; ++ch) F[ch] += w * d[ch];
                }
            }
            double* co = cn + ((size_t)r * W + q) * C;
            for (int ch = 0; ch < C; ++ch) co[ch] = ci[ch] + P->dt * P->s * F[ch];
        }
    }
    free(scratch);
    return OR_OK;
}

/* Forward sweep: traj holds K+1 fields, traj[0] = c0. */
int or_forward_sweep(const double* c0, int H, int W, int C, const or_params* P,
                     const double* eps, double* traj)
{
    const size_t n = (size_t)H * W * C;
    memcpy(traj, c0, n * sizeof(double));
    for (int k = 0; k < P->K; ++k) {
        int rc = or_forward_step(traj + (size_t)k * n, traj + (size_t)(k + 1) * n, H, W, C, P,
                                 eps[2 * k], eps[2 * k + 1]);
        if (rc) return rc;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Discrete adjoint of one Euler step (transpose of the Jacobian of      */
/* F, Sec. 3.1) plus the two control partials dl/d eps^k.                */
/*   p_i <- p_i + dt s sum_j [ phi (p_j - p_i)                           */
/*                            + ec phi' D_ij (D_ij . (p_j - p_i)) ]       */
/*   dl/d ex = dt s/2 sum_i sum_j phi' d2_ij   (p_i . D_ij)              */
/*   dl/d ec = dt s/2 sum_i sum_j phi' |D_ij|^2 (p_i . D_ij)             */
/* with D_ij = c_j - c_i, r and phi at (c^k, eps^k) and p = p^{k+1}.     */
int or_adjoint_step(const double* c, const double* p, double* pn, int H, int W, int C,
                    const or_params* P, double ex, double ec, double* gk /*[2]*/)
{
    const double dx = 1.0 / W, dy = 1.0 / H;
    const int R = P->R;
    /* per-row partial sums of the two control integrands, and per-row scratch
       (accumulator and differences of one pixel) */
    double* rowx = (double*)calloc((size_t)H, sizeof(double));
    double* rowc = (double*)calloc((size_t)H, sizeof(double));
    double* scratch = (double*)malloc(sizeof(double) * 2 * (size_t)H * (size_t)C);
    if (!rowx || !rowc || !scratch) {
        free(rowx);
        free(rowc);
        free(scratch);
        return OR_ENOMEM;
    }
#pragma omp parallel for schedule(static)
    for (int r = 0; r < H; ++r) {
        double* acc = scratch + 2 * (size_t)r * C;
        double* d = acc + C;
        double sx = 0.0, sc = 0.0;
        for (int q = 0; q < W; ++q) {
            const size_t i = ((size_t)r * W + q) * C;
            const double* ci = c + i;
            const double* pi = p + i;
            for (int ch = 0; ch < C; ++ch) acc[ch] = 0.0;
            for (int a = -R; a <= R; ++a) {
                int rr = r + a;
                if (rr < 0 || rr >= H) continue;
                for (int b = -R; b <= R; ++b) {
                    int qq = q + b;
                    if (qq < 0 || qq >= W) continue;
                    const size_t j = ((size_t)rr * W + qq) * C;
                    const double* cj = c + j;
                    const double* pj = p + j;
                    double d2 = (b * dx) * (b * dx) + (a * dy) * (a * dy);
                    double n2 = 0.0;
                    for (int ch = 0; ch < C; ++ch) {
                        d[ch] = cj[ch] - ci[ch];
                        n2 += d[ch] * d[ch];
                    }
                    double rij = 0.5 * ex * d2 + 0.5 * ec * n2;
                    double w = kern(P, rij);
                    double w1 = dkern(P, rij);
                    double ddp = 0.0, pid = 0.0;
                    for (int ch = 0; ch < C; ++ch) {
                        ddp += d[ch] * (pj[ch] - pi[ch]);
                        pid += pi[ch] * d[ch];
                    }
                    for (int ch = 0; ch < C; ++ch)
                        acc[ch] += w * (pj[ch] - pi[ch]) + ec * w1 * ddp * d[ch];
                    sx += w1 * d2 * pid;
                    sc += w1 * n2 * pid;
                }
            }
            for (int ch = 0; ch < C; ++ch) pn[i + ch] = pi[ch] + P->dt * P->s * acc[ch];
        }
        rowx[r] = sx;
        rowc[r] = sc;
    }
    double tx = 0.0, tc = 0.0;
    for (int r = 0; r < H; ++r) {
        tx += rowx[r];
        tc += rowc[r];
    }
    gk[0] = P->dt * 0.5 * P->s * tx;
    gk[1] = P->dt * 0.5 * P->s * tc;
    free(rowx);
    free(rowc);
    free(scratch);
    return OR_OK;
}

/* Adjoint sweep from p^K = pK back to p^0; geps[k*2+{0,1}] = dl/d eps^k. */
int or_adjoint_sweep(const double* traj, int H, int W, int C, const or_params* P,
                     const double* eps, const double* pK, double* p0, double* geps)
{
    const size_t n = (size_t)H * W * C;
    double* a = (double*)malloc(n * sizeof(double));
    double* b = (double*)malloc(n * sizeof(double));
    if (!a || !b) {
        free(a);
        free(b);
        return OR_ENOMEM;
    }
    memcpy(a, pK, n * sizeof(double));
    for (int k = P->K - 1; k >= 0; --k) {
        int rc = or_adjoint_step(traj + (size_t)k * n, a, b, H, W, C, P, eps[2 * k], eps[2 * k + 1],
                                 geps + 2 * k);
        if (rc) {
            free(a);
            free(b);
            return rc;
        }
        double* t = a;
        a = b;
        b = t;
    }
    memcpy(p0, a, n * sizeof(double));
    free(a);
    free(b);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Discrete gradient grad# (Def. 3.1) with the reflective boundary rule: */
/* at the first/last column (row) the reflected neighbour equals the     */
/* opposite one, so the central difference vanishes there.               */
void or_grad(const double* c, int H, int W, int C, double* g)
{
    const double dx = 1.0 / W, dy = 1.0 / H;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < H; ++r)
        for (int q = 0; q < W; ++q)
            for (int ch = 0; ch < C; ++ch) {
                double gx = 0.0, gy = 0.0;
                if (q >= 1 && q <= W - 2)
                    gx = (c[((size_t)r * W + q + 1) * C + ch] - c[((size_t)r * W + q - 1) * C + ch]) / (2.0 * dx);
                if (r >= 1 && r <= H - 2)
                    gy = (c[((size_t)(r + 1) * W + q) * C + ch] - c[((size_t)(r - 1) * W + q) * C + ch]) / (2.0 * dy);
                g[(((size_t)r * W + q) * 2 + 0) * C + ch] = gx;
                g[(((size_t)r * W + q) * 2 + 1) * C + ch] = gy;
            }
}

/* Divergence as the negative transpose of grad#:                       */
/* (div w)_{r,q} = (w^x_{r,q+1}[q+1 interior] - w^x_{r,q-1}[q-1 interior])/(2dx) */
/*               + (same along rows)/(2dy).                              */
void or_div(const double* w, int H, int W, int C, double* out)
{
    const double dx = 1.0 / W, dy = 1.0 / H;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < H; ++r)
        for (int q = 0; q < W; ++q)
            for (int ch = 0; ch < C; ++ch) {
                double v = 0.0;
                if (q + 1 >= 1 && q + 1 <= W - 2) v += w[(((size_t)r * W + q + 1) * 2 + 0) * C + ch] / (2.0 * dx);
                if (q - 1 >= 1 && q - 1 <= W - 2) v -= w[(((size_t)r * W + q - 1) * 2 + 0) * C + ch] / (2.0 * dx);
                if (r + 1 >= 1 && r + 1 <= H - 2) v += w[(((size_t)(r + 1) * W + q) * 2 + 1) * C + ch] / (2.0 * dy);
                if (r - 1 >= 1 && r - 1 <= H - 2) v -= w[(((size_t)(r - 1) * W + q) * 2 + 1) * C + ch] / (2.0 * dy);
                out[((size_t)r * W + q) * C + ch] = v;
            }
}

/* ------------------------------------------------------------------ */
/* Energies: TV and fidelity (eq. cost_TV), the regularised Lagrangian  */
/* L (eq. cost_tv_regular) and the completed square L~ (eq.              */
/* complete_square), plus the residual of v - grad c.                    */
int or_energies_eval(const double* c, const double* c0, const double* v, const double* mu,
                     int H, int W, int C, const or_params* P, or_energies* E)
{
    const size_t n2c = (size_t)H * W * 2 * C;
    const double dx = 1.0 / W, dy = 1.0 / H, area = dx * dy;
    double* g = (double*)malloc(n2c * sizeof(double));
    double* acc = (double*)calloc((size_t)H * 8, sizeof(double));
    if (!g || !acc) {
        free(g);
        free(acc);
        return OR_ENOMEM;
    }
    or_grad(c, H, W, C, g);
#pragma omp parallel for schedule(static)
    for (int r = 0; r < H; ++r) {
        double tv = 0, fid = 0, lsum = 0, lt = 0, svg = 0, sg = 0, sv = 0;
        for (int q = 0; q < W; ++q) {
            const size_t pix = (size_t)r * W + q;
            double ng = 0, nv = 0, nvg = 0, muvg = 0, nmu = 0, nsh = 0, nf = 0;
            for (int k = 0; k < 2 * C; ++k) {
                double gk = g[pix * 2 * C + k];
                double vk = v ? v[pix * 2 * C + k] : 0.0;
                double mk = mu ? mu[pix * 2 * C + k] : 0.0;
                ng += gk * gk;
                nv += vk * vk;
                nvg += (vk - gk) * (vk - gk);
                muvg += mk * (vk - gk);
                nmu += mk * mk;
                double sh = vk - gk + mk / P->rho;
                nsh += sh * sh;
            }
            for (int ch = 0; ch < C; ++ch) {
                double e = c[pix * C + ch] - c0[pix * C + ch];
                nf += e * e;
            }
            tv += sqrt(ng);
            fid += 0.5 * P->alpha * nf;
            lsum += sqrt(nv) + muvg + 0.5 * P->rho * nvg + 0.5 * P->alpha * nf;
            lt += 0.5 * P->rho * nsh + sqrt(nv) + 0.5 * P->alpha * nf;
            svg += nvg;
            sg += ng;
            sv += nv;
            (void)nmu;
        }
        acc[r * 8 + 0] = tv;
        acc[r * 8 + 1] = fid;
        acc[r * 8 + 2] = lsum;
        acc[r * 8 + 3] = lt;
        acc[r * 8 + 4] = svg;
        acc[r * 8 + 5] = sg;
        acc[r * 8 + 6] = sv;
    }
    double t[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int r = 0; r < H; ++r)
        for (int k = 0; k < 7; ++k) t[k] += acc[r * 8 + k];
    E->TV = area * t[0];
    E->fid = area * t[1];
    E->K = E->TV + E->fid;
    E->L = area * t[2];
    E->Ltilde = area * t[3];
    E->sq_vg = t[4];
    E->sq_g = t[5];
    E->sq_v = t[6];
    E->r_abs = sqrt(area * t[4]);
    double den = sqrt(t[5]);
    if (sqrt(t[6]) > den) den = sqrt(t[6]);
    if (den < 1e-30) den = 1e-30;
    E->r_rel = sqrt(t[4]) / den;
    free(g);
    free(acc);
    return OR_OK;
}

/* Completed-square objective L~(c, v) and its gradient in c            */
/* (eq. admm_terminal rewritten with div = -grad#^T):                    */
/*   dL~/dc = dx dy [ div(mu + rho (v - grad c)) + alpha (c - c0) ].     */
int or_terminal(const double* c, const double* c0, const double* v, const double* mu,
                int H, int W, int C, const or_params* P, double* pK, double* Ltilde)
{
    const size_t n = (size_t)H * W * C, n2c = 2 * n;
    const double area = (1.0 / W) * (1.0 / H);
    double* g = (double*)malloc(n2c * sizeof(double));
    double* qf = (double*)malloc(n2c * sizeof(double));
    double* dv = (double*)malloc(n * sizeof(double));
    int rc = OR_OK;
    if (!g || !qf || !dv) {
        rc = OR_ENOMEM;
        goto done;
    }
    or_grad(c, H, W, C, g);
    for (size_t k = 0; k < n2c; ++k) {
        double vk = v ? v[k] : 0.0, mk = mu ? mu[k] : 0.0;
        qf[k] = mk + P->rho * (vk - g[k]);
    }
    or_div(qf, H, W, C, dv);
    if (pK)
        for (size_t k = 0; k < n; ++k) pK[k] = area * (dv[k] + P->alpha * (c[k] - c0[k]));
    if (Ltilde) {
        or_energies E;
        rc = or_energies_eval(c, c0, v, mu, H, W, C, P, &E);
        if (rc == OR_OK) *Ltilde = E.Ltilde;
    }
done:
    free(g);
    free(qf);
    free(dv);
    return rc;
}

/* Shrinkage (eq. soft_threshold): per pixel, with a = grad c - mu/rho   */
/* taken jointly over all 2C components,                                  */
/*   v = (|a| - 1/rho) a/|a|  if |a| > 1/rho,  else 0.                    */
/* Then, if update_mu, the dual ascent of eq. dual_ascent:                */
/*   mu <- mu + gamma (v - grad c).                                       */
int or_pd_step(const double* c, const double* c0, int H, int W, int C, const or_params* P,
               double* v, double* mu, int update_mu, or_energies* E)
{
    const size_t npix = (size_t)H * W, n2c = npix * 2 * C;
    double* g = (double*)malloc(n2c * sizeof(double));
    if (!g) return OR_ENOMEM;
    or_grad(c, H, W, C, g);
    const double thr = 1.0 / P->rho;
#pragma omp parallel for schedule(static)
    for (long pix = 0; pix < (long)npix; ++pix) {
        double na = 0.0;
        for (int k = 0; k < 2 * C; ++k) {
            double a = g[pix * 2 * C + k] - mu[pix * 2 * C + k] / P->rho;
            na += a * a;
        }
        na = sqrt(na);
        for (int k = 0; k < 2 * C; ++k) {
            double a = g[pix * 2 * C + k] - mu[pix * 2 * C + k] / P->rho;
            v[pix * 2 * C + k] = (na > thr) ? (na - thr) * a / na : 0.0;
        }
        if (update_mu)
            for (int k = 0; k < 2 * C; ++k)
                mu[pix * 2 * C + k] += P->gamma * (v[pix * 2 * C + k] - g[pix * 2 * C + k]);
    }
    free(g);
    return E ? or_energies_eval(c, c0, v, mu, H, W, C, P, E) : OR_OK;
}

/* ------------------------------------------------------------------ */
/* Solver: method of multipliers (Alg. 2) whose control argmin is the    */
/* direct-adjoint loop with two-way projected Armijo search (Alg. 1,     */
/* terminal condition of eq. admm_terminal).                             */
/*                                                                       */
/* With P->cost == 1 the same DAL loop runs once on the quadratic cost   */
/* J of Def. 3.2 (Sec. 3.1): J(c) = dx dy sum [|grad c|^2 + alpha        */
/* (c - c0)^2] / 2 and dJ/dc = dx dy [-div grad c + alpha (c - c0)],     */
/* which is L~ and its gradient at v = mu = 0, rho = 1; there are no     */
/* v / mu updates.                                                       */
/*                                                                       */
/* decisions_in / decisions_out hold one double per DAL iteration, laid  */
/* out [max_outer][max_inner]: the accepted step tau (> 0), or 0 where   */
/* the inner loop ended without a step.  With decisions_in the search is */
/* replaced by the recorded steps (replay).  trace_out, when given, gets */
/* OR_TRACE doubles per DAL iteration: Phi before the step, Phi after it */
/* (0 when no step was taken), the number of trials, and the smallest   */
/* Armijo margin of those trials, min |Phi(0) + c <G, de> - Phi(tau)| /  */
/* |Phi(0)| (how far each sufficient-decrease test was from going the   */
/* other way; NaN when no trial ran).  eps_log and grad_log             */
/* ([max_outer][max_inner][K][2]) receive the controls after each        */
/* accepted step and the gradient G of each DAL iteration.               */
#define OR_TRACE 4

static double clampd(double x, double lo, double hi)
{
    return x < lo ? lo : (x > hi ? hi : x);
}

static void project_step(const double* eps, const double* G, double tau, const or_params* P,
                         double* out)
{
    for (int k = 0; k < P->K; ++k)
        for (int m = 0; m < 2; ++m)
            out[2 * k + m] = clampd(eps[2 * k + m] - tau * G[2 * k + m], P->eps_min[m], P->eps_max[m]);
}

/* One Armijo trial: eps(tau) = Pi_E(eps - tau G), forward sweep into traj,
   Phi(tau) = L~(c^K(tau)), and the projected sufficient-decrease test
   Phi(tau) <= Phi(0) + c <G, eps(tau) - eps>, with the rectangular-rule
   inner product dt * sum_k (Sec. 3.2).  *pass is 1 when the test passes;
   *margin (may be NULL) receives (Phi(0) + c <G, de> - Phi(tau)) / |Phi(0)|.
   Returns OR_OK or an error code. */
static int armijo_trial(const double* c0, int H, int W, int C, const or_params* P,
                        const double* v, const double* mu, const double* eps, const double* G,
                        double tau, double phi0, double* e_out, double* traj, double* phi_out,
                        int* pass, double* margin)
{
    const size_t n = (size_t)H * W * C;
    project_step(eps, G, tau, P, e_out);
    int rc = or_forward_sweep(c0, H, W, C, P, e_out, traj);
    if (rc) return rc;
    rc = or_terminal(traj + (size_t)P->K * n, c0, v, mu, H, W, C, P, NULL, phi_out);
    if (rc) return rc;
    double ip = 0.0;
    for (int k = 0; k < 2 * P->K; ++k) ip += G[k] * (e_out[k] - eps[k]);
    ip *= P->dt;
    const double rhs = phi0 + P->armijo_c * ip;
    *pass = *phi_out <= rhs;
    if (margin) *margin = (rhs - *phi_out) / fabs(phi0);
    return OR_OK;
}

int or_solve(const double* c0, int H, int W, int C, const or_params* P,
             double* eps /* [K*2] in/out */, double* mu /* [N*2C] in/out */,
             double* v /* [N*2C] out */, double* cK /* [N*C] out */,
             const double* decisions_in, double* decisions_out, double* trace_out,
             double* eps_log, double* grad_log, or_stats* st)
{
    if (!c0 || !eps || !mu || !v || !cK || H < 1 || W < 1 || C < 1 || P->K < 1 || P->R < 0 ||
        P->dt <= 0 || P->rho <= 0 || P->max_outer < 0 || P->max_inner < 0 || P->max_ls < 1)
        return OR_EINVAL;
    const int K = P->K;
    const size_t n = (size_t)H * W * C, fsz = n * (size_t)(K + 1);
    double* base = (double*)malloc(fsz * sizeof(double));
    double* cand = (double*)malloc(fsz * sizeof(double));
    double* trial = (double*)malloc(fsz * sizeof(double));
    double* pK = (double*)malloc(n * sizeof(double));
    double* p0 = (double*)malloc(n * sizeof(double));
    double* G = (double*)malloc(2 * (size_t)K * sizeof(double));
    double* e_try = (double*)malloc(2 * (size_t)K * sizeof(double));
    double* e_cand = (double*)malloc(2 * (size_t)K * sizeof(double));
    double* e_next = (double*)malloc(2 * (size_t)K * sizeof(double));
    int rc = OR_OK;
#define OR_TRY(expr)              \
    do {                          \
        if ((rc = (expr)) != 0)   \
            goto cleanup;         \
    } while (0)
    if (!base || !cand || !trial || !pK || !p0 || !G || !e_try || !e_cand || !e_next) {
        rc = OR_ENOMEM;
        goto cleanup;
    }
    or_stats S;
    memset(&S, 0, sizeof(S));
    const int quad = P->cost == 1;
    or_params Pq = *P;   /* parameters of the inner objective */
    if (quad) Pq.rho = 1.0;
    const double* tv = quad ? NULL : v;   /* v, mu seen by the inner objective */
    const double* tmu = quad ? NULL : mu;
    const int n_outer = quad ? (P->max_outer > 0 ? 1 : 0) : P->max_outer;
    if (decisions_out)
        for (int k = 0; k < P->max_outer * P->max_inner; ++k) decisions_out[k] = 0.0;
    if (trace_out)
        for (int k = 0; k < P->max_outer * P->max_inner; ++k) {
            trace_out[OR_TRACE * k + 0] = 0.0;
            trace_out[OR_TRACE * k + 1] = 0.0;
            trace_out[OR_TRACE * k + 2] = 0.0;
            trace_out[OR_TRACE * k + 3] = NAN;
        }
    const size_t nlog = (size_t)P->max_outer * P->max_inner * 2 * (size_t)P->K;
    if (eps_log) memset(eps_log, 0, nlog * sizeof(double));
    if (grad_log) memset(grad_log, 0, nlog * sizeof(double));

    double sigma = P->sigma0;
    /* Alg. 2: forward integration, then v^(0) = argmin_v L(c^(0), v, mu^(0)). */
    OR_TRY(or_forward_sweep(c0, H, W, C, P, eps, base));
    if (quad) {
        memset(v, 0, 2 * n * sizeof(double));
        memset(mu, 0, 2 * n * sizeof(double));
    } else {
        OR_TRY(or_pd_step(base + (size_t)K * n, c0, H, W, C, P, v, mu, 0, NULL));
    }
    double L_prev = NAN;
    int phi_seen = 0;
    or_energies E;
    memset(&E, 0, sizeof(E));

    for (int j = 0; j < n_outer; ++j) {
        /* control argmin: DAL iterations */
        for (int it = 0; it < P->max_inner; ++it) {
            const int slot = j * P->max_inner + it;
            double phi0;
            OR_TRY(or_terminal(base + (size_t)K * n, c0, tv, tmu, H, W, C, &Pq, pK, &phi0));
            if (!phi_seen) {
                S.phi_first = phi0;
                phi_seen = 1;
            }
            S.phi_last = phi0;
            OR_TRY(or_adjoint_sweep(base, H, W, C, P, eps, pK, p0, G));
            int all_zero = 1;
            for (int k = 0; k < 2 * K; ++k) {
                G[k] /= P->dt; /* L^2(0,T) gradient: dPhi/deps^k / dt */
                if (G[k] != 0.0) all_zero = 0;
            }
            S.inner_iters++;
            if (trace_out) trace_out[OR_TRACE * slot + 0] = phi0;
            if (grad_log) memcpy(grad_log + (size_t)slot * 2 * K, G, 2 * (size_t)K * sizeof(double));
            if (decisions_in && decisions_in[slot] <= 0.0) break;
            if (!decisions_in && all_zero) break;

            double accepted = 0.0, phi_acc = phi0;
            double margin = 0.0, min_margin = INFINITY;
            int ok = 0;
            if (decisions_in) {
                /* replayed step: one trial at the recorded tau, taken whatever its test says */
                accepted = decisions_in[slot];
                OR_TRY(armijo_trial(c0, H, W, C, &Pq, tv, tmu, eps, G, accepted, phi0, e_cand, cand,
                                    &phi_acc, &ok, &margin));
                min_margin = fabs(margin);
                S.ls_evals++;
            } else {
                /* Two-way search along the projected path (Alg. 1). */
                double tau = sigma, phit;
                int evals = 0, have = 0;
                OR_TRY(armijo_trial(c0, H, W, C, &Pq, tv, tmu, eps, G, tau, phi0, e_try, trial, &phit,
                                    &ok, &margin));
                evals++;
                min_margin = fabs(margin);
                if (ok) {
                    /* expanding branch: grow tau while the test keeps passing */
                    { double* t = cand; cand = trial; trial = t; }
                    memcpy(e_cand, e_try, 2 * (size_t)K * sizeof(double));
                    accepted = tau;
                    phi_acc = phit;
                    have = 1;
                    while (evals < P->max_ls) {
                        project_step(eps, G, tau / P->armijo_b, P, e_next);
                        if (memcmp(e_next, e_cand, 2 * (size_t)K * sizeof(double)) == 0)
                            break; /* the projected point no longer moves */
                        tau /= P->armijo_b;
                        OR_TRY(armijo_trial(c0, H, W, C, &Pq, tv, tmu, eps, G, tau, phi0, e_try, trial,
                                            &phit, &ok, &margin));
                        evals++;
                        if (fabs(margin) < min_margin) min_margin = fabs(margin);
                        if (!ok) break;
                        { double* t = cand; cand = trial; trial = t; }
                        memcpy(e_cand, e_try, 2 * (size_t)K * sizeof(double));
                        accepted = tau;
                        phi_acc = phit;
                    }
                } else {
                    /* backtracking branch: shrink tau until the test passes */
                    while (evals < P->max_ls) {
                        tau *= P->armijo_b;
                        OR_TRY(armijo_trial(c0, H, W, C, &Pq, tv, tmu, eps, G, tau, phi0, e_try, trial,
                                            &phit, &ok, &margin));
                        evals++;
                        if (fabs(margin) < min_margin) min_margin = fabs(margin);
                        if (ok) {
                            { double* t = cand; cand = trial; trial = t; }
                            memcpy(e_cand, e_try, 2 * (size_t)K * sizeof(double));
                            accepted = tau;
                            phi_acc = phit;
                            have = 1;
                            break;
                        }
                    }
                }
                S.ls_evals += evals;
                if (trace_out) trace_out[OR_TRACE * slot + 2] = evals;
                if (trace_out) trace_out[OR_TRACE * slot + 3] = min_margin;
                if (!have) break; /* no admissible step: the control argmin ends here */
                sigma = accepted;
            }
            /* accept: eps <- eps(sigma), trajectory <- that trial's */
            memcpy(eps, e_cand, 2 * (size_t)K * sizeof(double));
            { double* t = base; base = cand; cand = t; }
            if (decisions_out) decisions_out[slot] = accepted;
            if (trace_out) {
                trace_out[OR_TRACE * slot + 1] = phi_acc;
                trace_out[OR_TRACE * slot + 3] = min_margin;
            }
            if (eps_log) memcpy(eps_log + (size_t)slot * 2 * K, eps, 2 * (size_t)K * sizeof(double));
            /* relative stationarity of the inner objective (Rmk. on the convergence criteria) */
            if (P->tol_dal > 0.0 && fabs(phi_acc - phi0) < P->tol_dal * fabs(phi0)) break;
        }
        if (quad) {
            OR_TRY(or_energies_eval(base + (size_t)K * n, c0, NULL, NULL, H, W, C, &Pq, &E));
            S.outer_iters = 1;
            break;
        }
        /* v- and mu-updates (Alg. 2, eq. soft_threshold and eq. dual_ascent) */
        OR_TRY(or_pd_step(base + (size_t)K * n, c0, H, W, C, P, v, mu, 1, &E));
        S.outer_iters = j + 1;
        S.gap_rel = isnan(L_prev) ? NAN : fabs(E.L - L_prev) / fabs(L_prev);
        L_prev = E.L;
        if (P->tol_alm > 0.0 && E.r_rel < P->tol_alm) break;
        /* stop once the Lagrangian's change between multiplier iterations is small (Sec. 4.1) */
        if (P->tol_gap > 0.0 && !isnan(S.gap_rel) && S.gap_rel < P->tol_gap) break;
    }
    if (S.outer_iters == 0) OR_TRY(or_energies_eval(base + (size_t)K * n, c0, tv, tmu, H, W, C, &Pq, &E));
    memcpy(cK, base + (size_t)K * n, n * sizeof(double));
    S.K = E.K;
    S.TV = E.TV;
    S.fid = E.fid;
    S.L = E.L;
    S.Ltilde = E.Ltilde;
    S.r_rel = E.r_rel;
    S.r_abs = E.r_abs;
    S.status = (!quad && P->tol_alm > 0.0 && !(E.r_rel < P->tol_alm)) ? 1 : 0;
    if (st) *st = S;
cleanup:
#undef OR_TRY
    free(base); free(cand); free(trial); free(pK); free(p0); free(G);
    free(e_try); free(e_cand); free(e_next);
    return rc;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
