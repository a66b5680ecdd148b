/*
 * abc.h -- C ABI of the gfx950 (AMD Instinct MI355X) solver for the
 * agent-based optimal-control method of "Agent-Based Optimal Control for
 * Image Processing" (Oliviero, Cacace, Visconti, arXiv 2510.16154).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Arrays are FP32 and live in DEVICE memory unless marked "host".  The
 *    caller allocates all of them (inputs, outputs and the workspace); the
 *    library never allocates or frees memory the caller can see.
 *  - Colour fields are H x W x C, channel fastest ("HWC"), row 0 first in
 *    memory.  Two-vector fields (the splitting variable v, the multiplier
 *    mu, gradients) are H x W x 2 x C: component 0 along columns (x),
 *    component 1 along rows (y).  The paper orders rows bottom to top
 *    (Sec. 2); with rows in memory order the y-components of v and mu flip
 *    sign and nothing else changes.
 *  - Controls are K x 2: eps[2k] = eps_x on step k, eps[2k+1] = eps_c
 *    (piecewise constant in time).
 *  - Grid spacing dx = 1/W, dy = 1/H (Def. 3.1); positions are normalised.
 *  - Shapes: H, W >= 1, 1 <= C <= 64 and H * W * C <= 4e9 (every element
 *    index of a field fits 32 unsigned bits); larger images give ABC_EINVAL.
 *  - All work is ordered on `stream` (a hipStream_t; NULL = the null stream).
 *    Calls that return host scalars synchronise that stream.
 *  - Return value: ABC_OK (0), a negative error or a positive warning.
 *    Arguments are validated before anything is launched.  No C++ exception
 *    crosses this boundary.  abc_last_error() describes the last failure of
 *    the calling thread.
 *  - Adjoint sign: the library returns gradients (p = dl/dc), i.e. p is minus
 *    the adjoint state lambda of the paper's optimality system (Sec. 3.1).
 */
#ifndef ABC_H
#define ABC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ABC_OK 0
#define ABC_EINVAL (-1)     /* bad argument, size or workspace too small          */
#define ABC_EHIP (-2)       /* HIP runtime failure (message has the HIP error)    */
#define ABC_ENONFINITE (-3) /* NaN or Inf found in an input image or control      */
#define ABC_ENOCONV 1       /* warning: caps reached before tol_alm; outputs valid */

#define ABC_MAX_CHANNELS 64
/* Radius up to which a tile must fit the LDS (ABC_EINVAL otherwise).  Past it
 * (up to ABC_MAX_DIRECT_RADIUS) a tile whose halo still leaves 8 waves per CU
 * runs the LDS-tiled kernels, any other runs direct kernels that split each
 * 8 x 8 pixel block's window over 4 to 16 waves (the tile's shape then does not
 * matter): O(N (2R+1)^2) work per step, meant for small images, among them the
 * un-windowed sum of eq. MAsystem (a window that covers the image, with
 * s = 1/N). */
#define ABC_MAX_RADIUS 16
#define ABC_MAX_DIRECT_RADIUS 32767
/* abc_params.R value asking for the radius of the kernel's support: the
 * library takes, for each image, R* of abc_support_radius() with eps_x at the
 * box's lower bound eps_min[0].  Every pair with phi(r_ij) > 0 for any
 * control in the box then lies inside the window, so the window sum is the
 * un-windowed sum of eq. MAsystem for every admissible control.  Not taken by
 * abc_solve_batched. */
#define ABC_RADIUS_SUPPORT (-1)

/* Solver parameters.  abc_default_params() fills the paper's values
 * (Sec. 3.2: dt = 0.25, E = [2,1100]^2, eps0 = 57, sigma0 = 1, b = 1/2,
 * c = 1e-4; Sec. 4.2: rho = gamma = 1e-2). */
typedef struct abc_params {
    int32_t K;           /* explicit Euler steps (horizon T = K dt)                 */
    float dt;            /* time step                                               */
    int32_t R;           /* interaction window radius in pixels (square window), in
                            [0, ABC_MAX_DIRECT_RADIUS], or ABC_RADIUS_SUPPORT        */
    float inv_norm;      /* s scaling the interaction sum; 0 => 1/min(N,(2R+1)^2)  */
    float eps_min[2];    /* control box E = [eps_min, eps_max] per component       */
    float eps_max[2];
    float eps_init;      /* control used where eps is not supplied                  */
    float alpha;         /* fidelity weight                                         */
    float rho;           /* penalty of the splitting (eq. cost_tv_regular)          */
    float gamma;         /* multiplier ascent step (eq. dual_ascent)                */
    int32_t max_outer;   /* multiplier iterations M (Alg. 2)                        */
    int32_t max_inner;   /* DAL iterations per control argmin P (Alg. 1)            */
    int32_t max_ls;      /* cap on Armijo trials per DAL iteration                  */
    double tol_alm;      /* stop when r_rel < tol_alm; 0 => run max_outer           */
    double tol_dal;      /* stop the inner loop when |dPhi|/|Phi| < tol_dal; 0 => P */
    double sigma0;       /* initial Armijo step                                     */
    double armijo_b;     /* Armijo factor b in (0,1)                                */
    double armijo_c;     /* sufficient-decrease constant c in (0,1)                 */
    int32_t ckpt_every;  /* 0 => full trajectory; k > 0 => checkpoint every k steps  */
    int32_t tile_x;      /* interaction tile width in pixels; 0 => library default  */
    int32_t tile_y;      /* interaction tile height in pixels; 0 => library default.
                            A tile is valid when tile_y is a multiple of the pixels per
                            thread (2 for up to 4 channels, else 1) and the workgroup,
                            tile_x * tile_y / (pixels per thread) threads times the
                            lanes per pixel (C/8 rounded up for 16-64 channels at
                            R <= 3, else 1), is a whole number of 64-lane waves, at
                            most 256 threads (1024 with several lanes per pixel), and
                            fits in LDS; otherwise calls return ABC_EINVAL          */
    int32_t cost;        /* ABC_COST_TV or ABC_COST_QUADRATIC (see abc_solve)         */
    int32_t adj_tile_x;  /* adjoint tile width; 0 => tile_x (or library default)     */
    int32_t adj_tile_y;  /* adjoint tile height; 0 => tile_y (or library default)    */
    int32_t flags;       /* ABC_FLAG_* bits                                          */
    double stop_K;       /* > 0: also stop once K <= stop_K (checked after the starting
                            forward sweep and after every accepted DAL step)        */
    double tol_gap;      /* > 0: stop once |L_j - L_{j-1}| / |L_{j-1}| < tol_gap, the
                            change of the Lagrangian between multiplier iterations
                            (the ADMM stop of Sec. 4.1)                             */
} abc_params;

#define ABC_FLAG_NO_GRAPHS 1 /* launch every sweep step directly instead of replaying captured HIP graphs */
#define ABC_FLAG_AUTOTUNE 2  /* abc_solve_batched with no tile given: time the tile candidates on the batch's
                                largest image first (as abc_autotune) and use the fastest; the choice is kept
                                for the process per GPU architecture, C, R and size class.  Other entry
                                points ignore it */
#define ABC_FLAG_PERSISTENT 4 /* abc_solve_batched: each Euler step runs as a grid of as many workgroups as
                                 the GPU holds at once, taking the tiles of all images from per-step atomic
                                 counters, instead of one workgroup per tile.  Same results.  Other entry
                                 points ignore it */

#define ABC_COST_TV 0        /* TV + fidelity (eq. cost_TV), method of multipliers (Alg. 2)  */
#define ABC_COST_QUADRATIC 1 /* quadratic J (Def. 3.2), direct-adjoint loop alone (Alg. 1) */

/* Statistics of a solve or of one primal/dual update (host struct). */
typedef struct abc_stats {
    int32_t status;      /* ABC_OK or ABC_ENOCONV                                   */
    int32_t outer_iters; /* multiplier iterations run                               */
    int32_t inner_iters; /* DAL iterations run (adjoint sweeps)                     */
    int32_t ls_evals;    /* Armijo trials (forward sweeps after the first)          */
    double K;            /* TV + fidelity energy (eq. cost_TV)                      */
    double TV, fid;      /* its two parts                                           */
    double L;            /* regularised Lagrangian (eq. cost_tv_regular)            */
    double Ltilde;       /* completed square (eq. complete_square)                  */
    double r_rel;        /* |v - grad c| / max(|grad c|, |v|)                        */
    double r_abs;        /* sqrt(dx dy sum |v - grad c|^2)                           */
    double gap_rel;      /* |L_j - L_{j-1}| / |L_{j-1}| (NaN after one iteration)    */
    double phi_first;    /* inner objective at the first DAL iteration              */
    double phi_last;     /* inner objective at the last DAL iteration               */
    double K_start;      /* TV energy after the starting forward sweep (NaN unless stop_K > 0) */
    double ms_start;     /* milliseconds from the call to the end of that sweep     */
} abc_stats;

/* Workspace kinds for abc_workspace_bytes(). */
#define ABC_WS_SOLVE 0
#define ABC_WS_FORWARD 1
#define ABC_WS_ADJOINT 2
#define ABC_WS_PD 3

/* Library version, major*10000 + minor*100 + patch. */
int abc_version(void);

/* Description of the calling thread's last failure ("" if none).  Valid until
 * the next call on the same thread. */
const char* abc_last_error(void);

/* Fill *p with the paper's parameter values (see abc_params).  Host only.
 * K = 20, R = 2, alpha = 3000, M = 5, P = 50, max_ls = 40 are this library's
 * defaults where the paper gives none. */
int abc_default_params(abc_params* p);

/* Bytes of device workspace the entry point `kind` (ABC_WS_*) needs for an
 * H x W x C image under *p.  Host only; launches nothing. */
int abc_workspace_bytes(int kind, int H, int W, int C, const abc_params* p, size_t* bytes);

/* Radius of the kernel's support on an H x W image (Sec. 2, the ellipsoid of
 * influence; eq. kernel vanishes for r >= 1): r_ij <= 1 needs
 * eps_x/2 |x_j - x_i|^2 <= 1, i.e. a distance of at most sqrt(2 / eps_x) in
 * the unit square, so
 *   *R = min(ceil(sqrt(2 / eps_x_min) max(H, W)), max(H, W) - 1)
 * (the whole image when eps_x_min = 0).  Pixel spacing is 1/W across and 1/H
 * down, as in abc_forward_dynamics.  Returns ABC_EINVAL for H or W < 1, a
 * negative or NaN eps_x_min, or a NULL R.  Host only. */
int abc_support_radius(int H, int W, float eps_x_min, int32_t* R);

/* Number of trajectory slots abc_forward_dynamics writes: K + 1 when
 * p->ckpt_every == 0, else ceil(K / ckpt_every) + 1 (slot m holds the state
 * after min(m * ckpt_every, K) steps).  Host only. */
int abc_traj_slots(const abc_params* p, int* slots);

/* Forward dynamics (eq. MAsystem with the distance of eq. ellipsoid, the
 * Wendland kernel of eq. kernel, explicit Euler, Sec. 3.2):
 *   c_i <- c_i + dt s sum_{|a|,|b| <= R, j inside} phi(r_ij) (c_j - c_i),
 *   r_ij = eps_x/2 ((b dx)^2 + (a dy)^2) + eps_c/2 |c_j - c_i|^2,
 *   phi(r) = (1 + 4 r)(1 - r)^4 on [0,1], 0 beyond.
 * c0: H x W x C.  eps: K x 2.  traj: abc_traj_slots() fields of H x W x C;
 * slot 0 receives a copy of c0.  ws: ABC_WS_FORWARD bytes (may be 0 when
 * ckpt_every == 0).  Asynchronous. */
int abc_forward_dynamics(const float* c0, int H, int W, int C, const float* eps,
                         const abc_params* p, float* traj, void* ws, size_t ws_bytes,
                         void* stream);

/* Discrete adjoint of abc_forward_dynamics (transpose of each Euler step,
 * Jacobians of Sec. 3.1) and the gradient in the controls:
 *   p^k_i = p^{k+1}_i + dt s sum_j [ phi (p_j - p_i)
 *                                   + eps_c phi' D_ij (D_ij . (p_j - p_i)) ],
 *   dl/deps_x^k = dt s/2 sum_i sum_j phi' d_ij^2   (p_i . D_ij),
 *   dl/deps_c^k = dt s/2 sum_i sum_j phi' |D_ij|^2 (p_i . D_ij),
 * with D_ij = c^k_j - c^k_i, phi at (c^k, eps^k) and p = p^{k+1}.
 * traj: as written by abc_forward_dynamics with the same p (checkpointed
 * trajectories are recomputed segment by segment inside ws).  gK = dl/dc^K
 * (H x W x C).  g0 receives dl/dc^0 (may equal gK).  geps receives K x 2
 * values dl/deps^k.  ws: ABC_WS_ADJOINT bytes.  Asynchronous. */
int abc_adjoint_dynamics(const float* traj, int H, int W, int C, const float* eps,
                         const abc_params* p, const float* gK, float* g0, float* geps,
                         void* ws, size_t ws_bytes, void* stream);

/* abc_adjoint_dynamics for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments and results (bit for bit) as
 * abc_adjoint_dynamics, without ws / ws_bytes: the workspace (the two adjoint
 * ping-pong fields, the per-step control-gradient partials and, when
 * checkpointed, the recomputed segment) lives in a device array of
 * ABC_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  Nothing is allocated or freed by the call.  Every
 * call on a GPU shares that GPU's array, so calls that overlap on one GPU
 * (different streams or host threads) race: order them.  Returns ABC_EINVAL,
 * before any launch, when abc_workspace_bytes(ABC_WS_ADJOINT, ...) exceeds
 * ABC_NOALLOC_SCRATCH_BYTES (for example 3 channels at K = 50 fit up to about
 * 1.3 million pixels).  Asynchronous. */
#define ABC_NOALLOC_SCRATCH_BYTES (32u << 20)
int abc_adjoint_dynamics_noalloc(const float* traj, int H, int W, int C, const float* eps,
                                 const abc_params* p, const float* gK, float* g0, float* geps,
                                 void* stream);

/* Terminal condition of the adjoint for the completed-square functional
 * (eq. complete_square, eq. admm_terminal with div = -grad#^T):
 *   gK = dx dy [ div(mu + rho (v - grad# cK)) + alpha (cK - c0) ],
 * and, when Ltilde (host) is non-NULL, the value of L~(cK, v, mu).
 * cK, c0: H x W x C; v, mu: H x W x 2 x C (NULL = zero).  gK may be NULL
 * (objective only).  ws: ABC_WS_PD bytes.  Synchronises when Ltilde != NULL. */
int abc_pd_terminal(const float* cK, const float* c0, const float* v, const float* mu,
                    int H, int W, int C, const abc_params* p, float* gK, double* Ltilde,
                    void* ws, size_t ws_bytes, void* stream);

/* One primal/dual update of the splitting (Alg. 2, eq. soft_threshold and
 * eq. dual_ascent): with g = grad# cK and a = g - mu/rho per pixel over all
 * 2C components,
 *   v = (|a| - 1/rho) a/|a| if |a| > 1/rho, else 0;
 *   mu <- mu + gamma (v - g)             (only when update_mu != 0).
 * v, mu: H x W x 2 x C, updated in place (mu is read even when
 * update_mu == 0).  st (host, may be NULL) receives the energies and
 * residuals at (cK, v, mu) after the update; then the stream is
 * synchronised.  ws: ABC_WS_PD bytes. */
int abc_pd_step(const float* cK, const float* c0, int H, int W, int C, const abc_params* p,
                float* v, float* mu, int update_mu, abc_stats* st, void* ws, size_t ws_bytes,
                void* stream);

/* Optional record / replay of the control argmin for abc_solve (host arrays,
 * each may be NULL).  Slots are [max_outer][max_inner], one per DAL
 * iteration, in order.
 *   decisions_in:  accepted step tau to take in each slot instead of running
 *                  the line search; a slot <= 0 ends that inner loop.
 *   decisions_out: the accepted step of each slot of this run (0 = none).
 *   eps_replay:    [slots][K][2] controls to adopt after each accepted step
 *                  instead of Pi_E(eps - tau G) (needs decisions_in).  The
 *                  gradient is still computed and logged.
 *   grad_out:      [slots][K][2] control gradient G (FP64) of each DAL
 *                  iteration (dPhi/deps^k divided by dt).
 *   phi_out:       [slots][5] objective before the step, after it, trials,
 *                  TV energy K after the step, milliseconds since the call.
 *   outer_out:     [max_outer][4] after each multiplier iteration: K, L,
 *                  r_rel and the elapsed milliseconds since the call began.
 *   eps_out:       [slots][K][2] the controls Pi_E(eps - tau G) of each
 *                  accepted step, from this run's own gradient G and the
 *                  accepted tau; with eps_replay they are computed from the
 *                  replayed base controls and logged, not taken (0 where no
 *                  step was accepted). */
typedef struct abc_solve_log {
    const double* decisions_in;
    double* decisions_out;
    const double* eps_replay;
    double* grad_out;
    double* phi_out;
    double* outer_out;
    double* eps_out;
} abc_solve_log;

/* Full solve: method of multipliers (Alg. 2) whose control argmin is the
 * direct-adjoint loop with a two-way projected Armijo search (Alg. 1 with the
 * terminal condition above).  Returns the final colour field c(T) for the
 * optimised controls ("the quantised field").
 *   c0: H x W x C input image.
 *   eps: K x 2 controls in/out, or NULL (start from eps_init, not returned).
 *   mu: H x W x 2 x C multiplier in/out, or NULL (start from 0, not returned).
 *   v_out: H x W x 2 x C final splitting variable, or NULL.
 *   c_out: H x W x C final field.
 *   ws: ABC_WS_SOLVE bytes.  st: host, may be NULL.
 *   log: host, may be NULL (see abc_solve_log).
 * With p->cost == ABC_COST_QUADRATIC the direct-adjoint loop runs once (at
 * most max_inner iterations) on J(c) = dx dy/2 sum [|grad# c|^2 + alpha
 * (c - c0)^2] (Def. 3.2), whose adjoint terminal condition dJ/dc = dx dy
 * [-div grad# c + alpha (c - c0)] (Sec. 3.1) is the TV one at v = mu = 0 and
 * rho = 1; v and mu stay 0 and st->Ltilde reports J.
 * Returns ABC_OK, or ABC_ENOCONV when tol_alm > 0 was not reached within
 * max_outer iterations.  Synchronises the stream before returning. */
int abc_solve(const float* c0, int H, int W, int C, const abc_params* p, float* eps, float* mu,
              float* v_out, float* c_out, void* ws, size_t ws_bytes, void* stream, abc_stats* st,
              abc_solve_log* log);

/* One image of a batched solve: device pointers, sizes in pixels. */
typedef struct abc_image {
    const float* c0; /* H x W x C input                                       */
    float* c_out;    /* H x W x C final field                                 */
    float* eps;      /* K x 2 controls in/out, or NULL (start from eps_init)  */
    float* mu;       /* H x W x 2 x C multiplier in/out, or NULL (start at 0) */
    int32_t H, W;
} abc_image;

/* Tile autotuner.  Times the forward and adjoint interaction kernels for every
 * admissible tile shape on the image c0 (H x W x C, device) under p's window
 * radius and channel count, and writes the fastest shapes into p->tile_x/y
 * (forward) and p->adj_tile_x/y (adjoint).  Results do not depend on the tile
 * shape (each pixel sums its window in a fixed order), only the time does.
 *   cache_path (host, may be NULL): JSON file of earlier results keyed by GPU
 *     architecture, C, R, H and W; a hit skips the timing, a miss appends.
 *   ws: ABC_WS_TUNE bytes.  best_us (host, may be NULL): the two best
 *     per-launch times in microseconds (0 on a cache hit).
 * Synchronises the stream. */
#define ABC_WS_TUNE 4
int abc_autotune(const float* c0, int H, int W, int C, abc_params* p, const char* cache_path, void* ws,
                 size_t ws_bytes, void* stream, double* best_us);

/* Bytes of device workspace abc_solve_batched needs for n >= 1 images of
 * sizes H[i] x W[i] x C (ABC_EINVAL for n < 1 or a shape abc_solve would
 * reject).  Host only. */
int abc_workspace_bytes_batched(const int32_t* H, const int32_t* W, int n, int C, const abc_params* p,
                                size_t* bytes);

/* Solves n independent images of different sizes with the same parameters
 * (the method of abc_solve, same arithmetic per image).  The images advance in
 * lockstep rounds: each round launches one kernel per Euler step that covers
 * the tiles of every image still in that phase (terminal condition, adjoint
 * sweep, the next Armijo trial of every image that needs one, or the
 * multiplier update), so that small images share the GPU instead of running
 * one after another.  An image leaves the rounds when its own loops end.
 * p->stop_K is checked after every multiplier iteration here.
 *   imgs: host array of n descriptors.  C: channels (shared).
 *   st: host array of n stats (may be NULL).
 *   finish_ms: host array of n completion times in ms after the call began
 *     (may be NULL).
 *   Workspace: abc_workspace_bytes_batched() with the same flags (ABC_FLAG_AUTOTUNE
 *     asks for room for any tile the tuner may pick).
 *   logs: host array of n record / replay logs, one per image, with the
 *     meaning and sizes abc_solve gives them (may be NULL, and so may each
 *     array in them); outer_out's times are ms since this call began.
 * Returns ABC_OK, or ABC_ENOCONV when some image did not reach tol_alm;
 * ABC_EINVAL before any launch for n < 1, a NULL imgs, or an image whose
 * shape abc_solve would reject.  Synchronises the stream before returning. */
int abc_solve_batched(const abc_image* imgs, int n, int C, const abc_params* p, void* ws, size_t ws_bytes,
                      void* stream, abc_stats* st, double* finish_ms, const abc_solve_log* logs);

/* ---- Learned warm start ---------------------------------------------------
 * A convolutional encoder-decoder predicting a starting multiplier field mu0
 * (H x W x 2 x 3, inside the unit ball per pixel) and starting controls eps0
 * (K x 2, inside E) from an RGB image, to start abc_solve (Alg. 2) closer to
 * its end point.  Layers (3 x 3 convolutions, zero padding, ReLU):
 *   3->16 (full res), 2x2 average pool, 16->32, 32->64 (half res),
 *   2x nearest upsample concatenated with the first layer's output (80),
 *   80->32, 32->6 (full res); mu0 = z / max(1, |z|);
 *   eps0 = eps_min (eps_max / eps_min)^e, e = sigmoid(Wl mean(64-ch features) + bl)
 *   (the box E read on a log scale; calls return ABC_EINVAL unless
 *   0 < eps_min <= eps_max < inf).
 * Weights are an FP32 blob (layout: per conv layer W[9 Cin][Cout] with row
 * (kh*3 + kw)*Cin + ci, then b[Cout]; then Wl[64][2K], bl[2K]).  Convolutions
 * run as BF16 x BF16 -> FP32 on the matrix cores (operands rounded to BF16).
 * Images are B x H x W x 3 FP32 with H, W even. */

/* Number of FP32 parameters for K control steps (K <= 128).  Host only. */
int abc_wsnet_param_count(int K, size_t* n);

/* Workspace bytes for a batch (train != 0: forward + backward).  Host only. */
int abc_wsnet_workspace_bytes(int B, int H, int W, int K, int train, size_t* bytes);

/* mu0 (B x H x W x 6) and eps0 (B x K x 2, in p's box E).  Synchronises. */
int abc_wsnet_forward(const float* params, const float* x, int B, int H, int W, int K, const abc_params* p,
                      float* mu0, float* eps0, void* ws, size_t ws_bytes, void* stream);

/* Loss = mean_pixels |mu0 - mu_t|^2 + w_eps mean (e - e_t)^2 (e, e_t the controls
 * mapped to [0,1] by E on a log scale: e_t = log(eps_t / eps_min) /
 * log(eps_max / eps_min)) and its gradient in the parameters (grad, same
 * layout as params; overwritten).  Every eps_t must be positive and finite
 * (ABC_EINVAL before any launch).  loss (host) may be NULL; otherwise
 * synchronises. */
int abc_wsnet_loss_grad(const float* params, const float* x, const float* mu_t, const float* eps_t, int B, int H,
                        int W, int K, const abc_params* p, float w_eps, float* grad, double* loss, void* ws,
                        size_t ws_bytes, void* stream);

/* One Adam step (bias-corrected, step t >= 1) on n parameters.  Asynchronous. */
int abc_wsnet_adam(float* params, const float* grad, float* m, float* v, size_t n, int t, float lr, float b1,
                   float b2, float eps, void* stream);

/* Description of the calling thread's last warm-start failure. */
const char* abc_wsnet_last_error(void);

/* ---- Segmentation scores (Sec. 4.4) ---------------------------------------
 * The paper scores a processed image by labelling its segments with a
 * watershed at threshold 0.02 and computing on those labels the intra-region
 * variance IRV (over the original image), the inter-region contrast IRC (over
 * the processed image) and the validity score VS = IRV / IRC:
 *   IRV = (1/N) sum_j sum_{p in R_j} |c0_p - mean(c0 over R_j)|^2,
 *   IRC = min_{i<j} |mean(c over R_i) - mean(c over R_j)|,
 * with |.| the Euclidean norm over channels; labels without pixels are
 * ignored and IRC = VS = NaN when fewer than two labels hold pixels.
 *
 * The watershed (the paper names no variant) is the marker-based one defined
 * as a minimum spanning forest, whose result is unique:
 *   relief g2(p) = sum_ch gx^2 + gy^2, gx = (c(q+1) - c(q-1)) / 2 and
 *     gy = (c(r+1) - c(r-1)) / 2 (central differences of Def. 3.1 in pixel
 *     units, zero on the first/last column and row), in FP32 with, per
 *     channel in ascending order, g2 = fma(gx, gx, fma(gy, gy, g2));
 *   markers: 4-connected components of {g2 < theta * theta (FP32)}; if none,
 *     the pixel of least g2 (lowest index among ties);
 *   edges: 4-neighbour pairs ordered by (max(g2 p, g2 q), index), index 2p
 *     for (p, p+1) and 2p+1 for (p, p+W), p = r*W + q;
 *   each pixel takes the marker component of its tree in the minimum
 *     spanning forest relative to the markers; components are numbered
 *     0..k-1 in order of their smallest pixel index.
 * Cost: the pairwise IRC search is O(k^2) in the number of labels. */
typedef struct abc_seg_stats {
    int32_t k;        /* labels: watershed segments, or max(labels_in) + 1          */
    int32_t nonempty; /* labels holding at least one pixel                          */
    int32_t rounds;   /* flooding rounds of the forest construction (0 with labels_in) */
    int32_t reserved;
    double irv, irc, vs;
} abc_seg_stats;

/* Workspace bytes of abc_segment for an H x W x C image (H*W < 2^31).  Host only. */
int abc_segment_workspace_bytes(int H, int W, int C, size_t* bytes);

/* Labels and scores one image.
 *   c: processed field, c0: original image, both H x W x C FP32 device, HWC.
 *   theta: watershed threshold (the paper uses 0.02).
 *   labels_in: device H x W int32 labels in [0, H*W) to score instead of the
 *     watershed (theta and labels_out are then unused), or NULL.
 *   labels_out: device H x W int32 watershed labels, or NULL.
 *   stats: host output.
 * The per-label sums behind IRV and IRC are fixed-point integer sums, so
 * the scores are the same bits on every run.
 * Returns ABC_OK, ABC_EINVAL (bad argument, small workspace, label out of
 * range), ABC_ENONFINITE (c or c0 holds a NaN or an infinity; nothing is
 * labelled) or ABC_EHIP.  Synchronises the stream (several times: the forest
 * is built in rounds whose count is read back). */
int abc_segment(const float* c, const float* c0, int H, int W, int C, float theta, const int32_t* labels_in,
                int32_t* labels_out, abc_seg_stats* stats, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ABC_H */
