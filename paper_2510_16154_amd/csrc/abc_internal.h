// Internal interface between the host solver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace abc {

// Records the calling thread's last error (returned by abc_last_error).
void set_last_error(const std::string& msg);

// Tile of pixels handled by one workgroup of the windowed interaction kernels
// (one or two pixels per thread, see rows_per_thread; the workgroup stages the
// tile plus an R-pixel halo in LDS).
struct Tile {
    int tx, ty;
};

// One image of a multi-image interaction launch.  The grid covers the tiles of
// all jobs; `start` is the job's first global tile.  Forward step k reads trajectory
// slot k and writes slot k+1; transposed step k reads slot k and ping-pongs
// between pa and pb (p^{k+1} in pa when K-1-k is even), writing its control
// partials to part + k * tiles * 2.
struct StepJob {
    float* traj;
    const float* eps;
    float* pa;
    float* pb;
    double* part;
    int H, W, tiles_x, tiles, start;
    float dts, dx2, dy2;
};

// One image of a multi-image per-pixel launch (256 pixels per block);
// `start` is the job's first global block.
struct PixJob {
    const float* c;
    const float* c0;
    float* v;
    float* mu;
    float* pK;
    float* part;
    int H, W, start;
    float area, inv2dx, inv2dy;
};

// One job of a multi-image reduction: rows x nblk partials (FP64 or FP32);
// FP64 results are multiplied by `scale`.
struct RedJob {
    const double* part_d;
    double* out_d;
    const float* part_f;
    float* out_f;
    double scale;
    int rows, nblk;
};

// Number of workgroups (= tiles) covering an H x W image.
int tile_count(int H, int W, Tile t);

// LDS bytes of one interaction workgroup (fields = 1 forward, 2 adjoint).
size_t tile_lds_bytes(int C, int R, Tile t, int fields);

// Default tile for (C, R) and kernel kind (fields = 1 forward, 2 adjoint).
Tile default_tile(int C, int R, int fields);

// Pixels each thread of the interaction kernels computes (vertically adjacent):
// 2 for 1 to 4 channels, else 1 (the wide kernels spread one pixel over lanes).  A tile of tx x ty
// pixels runs as tx x ty / rows_per_thread threads (times the lanes per pixel
// of the wide kernels).
int rows_per_thread(int C, int R);

// True when the (C, R, tile) combination fits the hardware limits: ty a
// multiple of rows_per_thread, a whole number of 64-lane waves, at most 256
// threads (1024 for the wide kernels) and the LDS budget (past ABC_MAX_RADIUS any
// such tile: one whose halo does not fit runs the direct kernels instead).
bool tile_ok(int C, int R, Tile t, int fields);

// True when a step of radius R with this tile runs the direct kernels: R past
// ABC_MAX_RADIUS and the tile's halo leaving fewer than 8 waves per CU (none
// when it does not fit the LDS).
bool direct_step(int C, int R, Tile t, int fields);

// Workgroups (8 x 8 pixel blocks) of a direct step on an H x W image.
int direct_blocks(int H, int W);

// Control-gradient partial slots per step of the transposed sweep with adjoint
// tile t: one per tile, or one per 8 x 8 block when the step runs direct.
int adj_part_count(int H, int W, int C, int R, Tile t);

// One explicit Euler step of the agent dynamics: cout = cin + dts * F(cin, eps^k).
// eps points to the K x 2 device control array; step k reads eps[2k], eps[2k+1].
hipError_t launch_forward_step(const float* cin, float* cout, const float* eps, int k, int H, int W,
                               int C, int R, float dts, Tile t, hipStream_t s);

// Transposed Euler step: pout = pin + dts * (dF/dc)^T pin at (c, eps^k), and per
// workgroup FP64 partial sums of the two control-gradient integrands written to
// part[2*tile + {0,1}] (raw sums of d^2 q and |D|^2 q, q = (phi'/20)(D . dp)).
hipError_t launch_adjoint_step(const float* c, const float* pin, float* pout, const float* eps, int k,
                               int H, int W, int C, int R, float dts, Tile t, double* part,
                               hipStream_t s);

// FP64 version of launch_reduce_rows; out (FP64) and out_f (FP32) may be NULL.
hipError_t launch_reduce_rows_f64(const double* part, int nrows, int nblk, int nq, double scale,
                                  double* out, float* out_f, hipStream_t s);

// out[r*nq + q] = scale * sum_i part[(r*nblk + i)*nq + q] for r < nrows, q < nq
// (strided per-thread sums, then the workgroup tree).
hipError_t launch_reduce_rows(const float* part, int nrows, int nblk, int nq, float* out, float scale,
                              hipStream_t s);

// Workgroups used by the per-pixel primal/dual kernels.
int pd_blocks(int H, int W);

// Terminal condition and objective partials: kTermQuantities floats per workgroup in
// part (objective, |grad c|, |c - c0|^2).
constexpr int kTermQuantities = 3;
hipError_t launch_terminal(const float* c, const float* c0, const float* v, const float* mu, int H,
                           int W, int C, float rho, float alpha, float area, float* pK, float* part,
                           hipStream_t s);

// Shrinkage / multiplier update with 7 partial sums per workgroup in part:
// |v-g|^2, |g|^2, |v|^2, |g|, |c-c0|^2, |v| + mu.(v-g), rho/2|v-g+mu/rho|^2 + |v|.
constexpr int kPdQuantities = 7;
hipError_t launch_pd_step(const float* c, const float* c0, float* v, float* mu, int update_mu, int H,
                          int W, int C, float rho, float gamma, float* part, hipStream_t s);

// Multi-image launches (jobs in device memory, sorted by start).  queue == NULL:
// one workgroup per tile.  Otherwise the persistent form: persistent_grid()
// workgroups take the tiles from 8 counters per step, queue[8 k .. 8 k + 7],
// which must hold 0 when step k starts.  Both forms give the same bits.
int persistent_grid(int C, int R, Tile t, int fields, int total);
hipError_t launch_forward_step_batched(const StepJob* jobs, int njobs, int total_tiles, int k, int C, int R, Tile t,
                                       int* queue, hipStream_t s);
hipError_t launch_adjoint_step_batched(const StepJob* jobs, int njobs, int total_tiles, int k, int K, int C, int R,
                                       Tile t, int* queue, hipStream_t s);
hipError_t launch_terminal_batched(const PixJob* jobs, int njobs, int total_blocks, int C, float rho, float alpha,
                                   hipStream_t s);
hipError_t launch_pd_step_batched(const PixJob* jobs, int njobs, int total_blocks, int update_mu, int C, float rho,
                                  float gamma, hipStream_t s);
// FP64: out_d[r*nq+q] = scale * sum over the job's row r; FP32: out_f[q] = sum (rows = 1).
hipError_t launch_reduce_jobs_f64(const RedJob* jobs, int njobs, int max_rows, int nq, hipStream_t s);
hipError_t launch_reduce_jobs(const RedJob* jobs, int njobs, int nq, hipStream_t s);

// Sets *flag (device int) to nonzero when x[0..n) holds a NaN or an Inf.
hipError_t launch_nonfinite(const float* x, size_t n, int* flag, hipStream_t s);

}  // namespace abc
