// gfx950 kernels of the agent-based optimal-control solver.
//
// Windowed interaction (forward Euler step of eq. MAsystem and its transpose,
// Sec. 3.1): one workgroup per tile, one or two vertically adjacent pixels
// per thread (two for up to 4 channels).  The workgroup
// stages its tile plus an R-pixel halo in LDS (channel-interleaved 16-byte
// slots with one extra value per pixel that is 1 inside the image and 0 for
// halo cells beyond the border), then every thread sums its (2R+1)^2 window in
// a fixed offset order
// (a = -R..R outer, b = -R..R inner, self skipped).  Each output therefore
// depends only on its own window and not on the tile shape.  Workgroups whose
// halo lies inside the image skip the border mask.
//
// The Wendland kernel is evaluated through t = clamp(1 - r, 0, 1):
//   phi  = (1 + 4r)(1 - r)^4 = (5 - 4t) t^4,
//   phi' = -20 r (1 - r)^3   = 20 (t - 1) t^3,
// and t itself comes from one fused multiply-add per neighbour,
//   t = clamp(om_ab - eps_c/2 |D|^2),  om_ab = 1 - eps_x/2 ((b dx)^2 + (a dy)^2).
//
// Reductions are deterministic: butterfly sums inside a wavefront, then a
// fixed-order sum over the wavefronts of a workgroup, then a tree over
// workgroups in a second kernel.  No floating-point atomics anywhere.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <type_traits>

#include "../../include/abc.h"
#include "abc_internal.h"

namespace abc {

namespace {

constexpr int kWave = 64;
constexpr int kMaxThreads = 256;
constexpr size_t kMaxLds = 160 * 1024;

__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum of v over the workgroup, valid in thread 0.  `red` holds >= 16 floats.
__device__ __forceinline__ float block_sum(float v, float* red) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nthreads = blockDim.x * blockDim.y;
    v = wave_sum(v);
    const int w = tid / kWave;
    if ((tid % kWave) == 0) red[w] = v;
    __syncthreads();
    float s = 0.0f;
    if (tid == 0) {
        const int nw = (nthreads + kWave - 1) / kWave;
        for (int i = 0; i < nw; ++i) s += red[i];
    }
    __syncthreads();
    return s;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// FP64 sum of v over the workgroup, valid in thread 0.  `red` holds >= 16 doubles.
__device__ __forceinline__ double block_sum_f64(double v, double* red) {
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    v = wave_sum_f64(v);
    const int w = tid / kWave;
    if ((tid % kWave) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0) {
        const int nw = (nthreads + kWave - 1) / kWave;
        for (int i = 0; i < nw; ++i) s += red[i];
    }
    __syncthreads();
    return s;
}

// Two block sums at once (the same sums, in the same order, as two calls of
// block_sum_f64), with one pair of barriers; red holds 2 doubles per wave.
__device__ __forceinline__ void block_sum2_f64(double& a, double& b, double* red) {
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    a = wave_sum_f64(a);
    b = wave_sum_f64(b);
    const int w = tid / kWave, nw = (nthreads + kWave - 1) / kWave;
    if ((tid % kWave) == 0) {
        red[w] = a;
        red[nw + w] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
    if (tid == 0) {
        for (int i = 0; i < nw; ++i) sa += red[i];
        for (int i = 0; i < nw; ++i) sb += red[nw + i];
    }
    __syncthreads();
    a = sa;
    b = sb;
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous run of tiles so that neighbouring tiles share halo data in the
// same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    const int per = nb / 8, rem = nb % 8;
    const int x = bid % 8, idx = bid / 8;
    return x < rem ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

// The interaction tile of a workgroup in a one-image launch, whose grid is
// (64 bh, strips) with bh = ceil(tiles_y / 8): the 8 XCDs take the workgroups
// round-robin in linear order, so XCD x = blockIdx.x % 8 gets band x of bh tile
// rows, and within its band visits column strips kStrip tiles wide
// (blockIdx.y), each row by row from the top ((blockIdx.x / 8) % kStrip is the
// column in the strip, blockIdx.x / 64 the row in the band).  The tile below a
// tile then comes kStrip tiles later and finds the halo rows they share in the
// XCD's L2; in row-major order it came a whole tile row later, too late on wide
// images.  Shifts and masks only: integer division costs tens of instructions
// per wave.  Returns false for workgroups past the last tile row or column.
constexpr int kStrip = 8;
__device__ __forceinline__ bool strip_tile(int tiles_x, int tiles_y, int& tcol, int& trow) {
    const int bh = (tiles_y + 7) >> 3;
    tcol = blockIdx.y * kStrip + ((blockIdx.x >> 3) & (kStrip - 1));
    trow = (blockIdx.x & 7) * bh + (blockIdx.x >> 6);
    return tcol < tiles_x && trow < tiles_y;
}

// LDS slot of one pixel: CP channels, then the inside mask, in whole 16-byte
// vectors (8 bytes for one channel) so that a neighbour is read with
// ds_read_b128 / b64.  The slot stride is an odd number of vectors: the
// lanes of a read then fall on distinct bank groups (an even stride such as
// 8 vectors for 31 channels would put every lane of a wave on the same banks).
template <int CP>
struct Slot {
    static constexpr int NV = CP == 1 ? 1 : (CP + 1 + 3) / 4;        // vectors holding data
    static constexpr int NS = CP == 1 ? 1 : (NV % 2 ? NV : NV + 1);  // vectors per slot (stride)
    static constexpr int CS = CP == 1 ? 2 : 4 * NS;                  // floats per slot
};

// Pixels per thread of the one-lane interaction kernels: two vertically
// adjacent pixels for up to 4 channels (any radius), one for wider pixels.
template <int CP>
struct RowsPerThread {
    static constexpr int value = CP <= 4 ? 2 : 1;
};

// Thread layers of the transposed step: with up to 4 channels and a compile-time
// radius each pixel's window is split by rows over two threads (blockDim.z = 2),
// which doubles the waves of a workgroup; small images have too few tiles to give
// a CU more than two workgroups, and two waves per SIMD leave most FP32
// instructions unpaired.
template <int CP, int RT>
struct AdjSplit {
    static constexpr int value = CP <= 4 && RT >= 1 ? 2 : 1;
};

template <int CP>
__device__ __forceinline__ void load_px(const float* p, float (&v)[CP], float& m) {
    if constexpr (CP == 1) {
        const float2 x = *reinterpret_cast<const float2*>(p);
        v[0] = x.x;
        m = x.y;
    } else {
        constexpr int NV = Slot<CP>::NV;
        float t[4 * NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const float4 x = reinterpret_cast<const float4*>(p)[i];
            t[4 * i + 0] = x.x;
            t[4 * i + 1] = x.y;
            t[4 * i + 2] = x.z;
            t[4 * i + 3] = x.w;
        }
#pragma unroll
        for (int ch = 0; ch < CP; ++ch) v[ch] = t[ch];
        m = t[CP];
    }
}

// Stage rows [y0-R, y0+TY+R) x cols [x0-R, x0+TX+R) of a HWC field into LDS
// slots; channels >= C and cells outside the image are 0, the mask slot is 1
// inside the image and 0 outside.  Loads carry no branches: every cell reads
// the image pixel nearest to it (row and column clamped into the image, so
// every address lies in the field; lanes past the staged block read its last
// row or column, so no load leaves the block's own cache lines) and the values
// of cells outside the image are replaced by 0 afterwards.  Element indices are 32-bit (H W C is at most
// 4e9); with C == CP the channel offsets are constants of the load
// instructions, otherwise they are clamped into the pixel.  Each pass has the
// loads of up to 2 RU cells (RU rows x two columns) in flight before it
// writes LDS; with NF = 2 it stages two fields of the same image (dst1 from
// src1) in the same passes, so that their loads are in flight together.
template <int CP, bool EXACT, int NF, int RU>
__device__ __forceinline__ void stage_cells(float* dst0, const float* __restrict__ src0, float* dst1,
                                            const float* __restrict__ src1, int H, int W, int C, int x0, int y0,
                                            int R, int LW, int LH) {
    // rows are dealt out over every layer of the workgroup (blockDim.z > 1 in the split transposed step)
    const int tyz = threadIdx.y + blockDim.y * threadIdx.z, byz = blockDim.y * blockDim.z;
    constexpr int NV = Slot<CP>::NV, CS = Slot<CP>::CS, NC = 2 * RU;
    const unsigned WC = (unsigned)W * (unsigned)C;
    for (int ly0 = tyz; ly0 < LH; ly0 += RU * byz) {
        unsigned rbase[RU];
        bool row_in[RU];
#pragma unroll
        for (int v = 0; v < RU; ++v) {
            // rows past the tile (no cell of theirs is written) read its last row
            const int gy = y0 - R + min(ly0 + v * (int)byz, LH - 1);
            const int gyc = min(max(gy, 0), H - 1);
            row_in[v] = gy == gyc;
            rbase[v] = (unsigned)gyc * WC;
        }
        for (int lx0 = threadIdx.x; lx0 < LW; lx0 += 2 * blockDim.x) {
            float t[NF][NC][CS];
            bool act[NC];
            int cell[NC];
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                const int ly = ly0 + (u >> 1) * byz, lx = lx0 + (u & 1) * blockDim.x;
                act[u] = ly < LH && lx < LW;
                cell[u] = ly * LW + lx;
                const int gx = x0 - R + min(lx, LW - 1);
                const int gxc = min(max(gx, 0), W - 1);
                const bool in = act[u] && row_in[u >> 1] && gx == gxc;
                const unsigned col = EXACT ? (unsigned)gxc * (unsigned)CP : (unsigned)gxc * (unsigned)C;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const float* s = (f == 0 ? src0 : src1) + (rbase[u >> 1] + col);
#pragma unroll
                    for (int ch = 0; ch < CS; ++ch) {
                        const float x = ch < CP ? s[EXACT ? ch : min(ch, C - 1)] : 0.0f;
                        t[f][u][ch] = (in && ch < CP && (EXACT || ch < C)) ? x : 0.0f;
                    }
                    t[f][u][CP] = in ? 1.0f : 0.0f;
                }
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
#pragma unroll
                for (int u = 0; u < NC; ++u) {
                    if (!act[u]) continue;
                    float* d = (f == 0 ? dst0 : dst1) + cell[u] * CS;
                    if constexpr (CP == 1) {
                        *reinterpret_cast<float2*>(d) = make_float2(t[f][u][0], t[f][u][1]);
                    } else {
#pragma unroll
                        for (int i = 0; i < NV; ++i)
                            reinterpret_cast<float4*>(d)[i] = make_float4(t[f][u][4 * i], t[f][u][4 * i + 1],
                                                                          t[f][u][4 * i + 2], t[f][u][4 * i + 3]);
                    }
                }
            }
        }
    }
}

// One field: four rows x two columns per pass for up to 4 channels (a 32 x 16
// tile and its halo of 5 in one pass of 256 threads), two rows for wider pixels.
template <int CP>
__device__ __forceinline__ void stage_tile(float* dst, const float* __restrict__ src, int H, int W, int C,
                                           int x0, int y0, int R, int LW, int LH) {
    constexpr int RU = CP <= 4 ? 4 : 2;
    if (C == CP)
        stage_cells<CP, true, 1, RU>(dst, src, nullptr, nullptr, H, W, C, x0, y0, R, LW, LH);
    else
        stage_cells<CP, false, 1, RU>(dst, src, nullptr, nullptr, H, W, C, x0, y0, R, LW, LH);
}

// Two fields of one image (the transposed step's c^k and p^{k+1}): staged in
// the same passes for up to 4 channels (8 cells' loads in flight per thread),
// one after the other for wider pixels, whose cells take more registers.
template <int CP>
__device__ __forceinline__ void stage_tile2(float* dst0, const float* __restrict__ src0, float* dst1,
                                            const float* __restrict__ src1, int H, int W, int C, int x0, int y0,
                                            int R, int LW, int LH) {
    if constexpr (CP <= 4) {
        if (C == CP)
            stage_cells<CP, true, 2, 2>(dst0, src0, dst1, src1, H, W, C, x0, y0, R, LW, LH);
        else
            stage_cells<CP, false, 2, 2>(dst0, src0, dst1, src1, H, W, C, x0, y0, R, LW, LH);
    } else {
        stage_tile<CP>(dst0, src0, H, W, C, x0, y0, R, LW, LH);
        stage_tile<CP>(dst1, src1, H, W, C, x0, y0, R, LW, LH);
    }
}

// Offset constants of a window of radius RT, written by the threads of a
// workgroup: om[a][b] = 1 - Ax b^2 - Ay a^2 (Ax = eps_x/2 dx^2, Ay = eps_x/2
// dy^2), in the operation order of the window loop.  (In the transposed step
// the same table measured slower than recomputing, so it is used only here.)
__device__ __forceinline__ void offset_table(float* om, int RT, float Ax, float Ay) {
    const int D = 2 * RT + 1;
    for (int i = threadIdx.x + threadIdx.y * blockDim.x; i < D * D; i += blockDim.x * blockDim.y) {
        const int a = i / D - RT, b = i % D - RT;
        om[i] = fmaf(-Ax, (float)(b * b), fmaf(-Ay, (float)(a * a), 1.0f));
    }
}

// ----------------------------------------------------------------------------
// Forward step.
// With a compile-time radius the offset constants om_ab come from a table in
// LDS (filled once per workgroup with the same expression), which takes one
// VALU operation per neighbour off the inner loop.  For up to 4 channels each
// thread computes NP = 2 vertically adjacent pixels: a neighbour read from
// LDS serves every pixel of the thread whose window holds it (the windows of
// rows y and y+1 share 2R of their 2R+1 rows).  Each pixel still sums its own
// window in the (a, b) order, so the result is the same bit for bit as with
// one pixel per thread.
template <int CP, int RT, int NP, bool BORDER>
__device__ __forceinline__ void fwd_window(const float* me, int LW, int R, const float (&ci)[NP][CP],
                                           float (&acc)[NP][CP], float Ax, float Ay, float ech, const float* omt) {
    constexpr int CS = Slot<CP>::CS;
    const int RR = RT > 0 ? RT : R;
    // r: row of the neighbour relative to the thread's first pixel; pixel m sees it at a = r - m
#pragma unroll
    for (int r = -RR; r <= RR + NP - 1; ++r) {
        const float* row = me + r * LW * CS;
#pragma unroll
        for (int b = -RR; b <= RR; ++b) {
            float cj[CP], mj;
            load_px<CP>(row + b * CS, cj, mj);
#pragma unroll
            for (int m = 0; m < NP; ++m) {
                const int a = r - m;
                if (a < -RR || a > RR || (a == 0 && b == 0)) continue;
                const float om = RT > 0 ? omt[(a + RR) * (2 * RR + 1) + b + RR]
                                        : fmaf(-Ax, (float)(b * b), fmaf(-Ay, (float)(a * a), 1.0f));
                float d[CP];
                float n2 = 0.0f;
#pragma unroll
                for (int ch = 0; ch < CP; ++ch) {
                    d[ch] = cj[ch] - ci[m][ch];
                    n2 = fmaf(d[ch], d[ch], n2);
                }
                const float t = clamp01(fmaf(-ech, n2, om));
                const float t2 = t * t;
                float w = fmaf(-4.0f, t, 5.0f) * (t2 * t2);
                if (BORDER) w *= mj;
#pragma unroll
                for (int ch = 0; ch < CP; ++ch) acc[m][ch] = fmaf(w, d[ch], acc[m][ch]);
            }
        }
    }
}

// One interaction tile of a forward step: stage, then NP pixels per thread
// (the workgroup is TX x TY/NP threads for a TX x TY tile).
template <int CP, int RT>
__device__ __forceinline__ void fwd_tile(const float* __restrict__ cin, float* __restrict__ cout, float exh,
                                         float ech, int H, int W, int C, int R, int tcol, int trow, float dts,
                                         float dx2, float dy2, float* lds) {
    constexpr int CS = Slot<CP>::CS;
    constexpr int NP = RowsPerThread<CP>::value;
    const int TX = blockDim.x, TY = NP * blockDim.y;
    const int x0 = tcol * TX, y0 = trow * TY;
    const int LW = TX + 2 * R, LH = TY + 2 * R;
    const bool interior = x0 >= R && y0 >= R && x0 + TX + R <= W && y0 + TY + R <= H;
    float* omt = lds + LW * LH * CS;
    if constexpr (RT > 0) offset_table(omt, RT, exh * dx2, exh * dy2);
    stage_tile<CP>(lds, cin, H, W, C, x0, y0, R, LW, LH);
    __syncthreads();
    const int gx = x0 + threadIdx.x, gy = y0 + NP * threadIdx.y;
    if (gx >= W || gy >= H) return;
    const float* me = lds + ((NP * threadIdx.y + R) * LW + threadIdx.x + R) * CS;
    float ci[NP][CP], acc[NP][CP], mi;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        load_px<CP>(me + m * LW * CS, ci[m], mi);
#pragma unroll
        for (int ch = 0; ch < CP; ++ch) acc[m][ch] = 0.0f;
    }
    if (interior)
        fwd_window<CP, RT, NP, false>(me, LW, R, ci, acc, exh * dx2, exh * dy2, ech, omt);
    else
        fwd_window<CP, RT, NP, true>(me, LW, R, ci, acc, exh * dx2, exh * dy2, ech, omt);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        if (gy + m >= H) break;
        float* o = cout + ((size_t)(gy + m) * W + gx) * C;
#pragma unroll
        for (int ch = 0; ch < CP; ++ch)
            if (ch < C) o[ch] = fmaf(dts, acc[m][ch], ci[m][ch]);
    }
}

template <int CP, int RT>
__global__ void __launch_bounds__(kMaxThreads)
fwd_step_kernel(const float* __restrict__ cin, float* __restrict__ cout, const float* __restrict__ eps,
                int k, int H, int W, int C, int Rrt, int tiles_x, int tiles_y, float dts, float dx2, float dy2) {
    extern __shared__ __align__(16) float lds[];
    const int R = RT > 0 ? RT : Rrt;
    int tcol, trow;
    if (!strip_tile(tiles_x, tiles_y, tcol, trow)) return;
    fwd_tile<CP, RT>(cin, cout, 0.5f * eps[2 * k], 0.5f * eps[2 * k + 1], H, W, C, R, tcol, trow, dts, dx2, dy2,
                     lds);
}

// Index of the last job whose first tile (or block) is <= g (jobs sorted by start).
template <class J>
__device__ __forceinline__ int find_job(const J* __restrict__ jobs, int njobs, int g) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].start <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Runs body(g) for the global tiles g of a multi-image launch.  Without a
// queue (PQ false) the grid has one workgroup per tile, handed to the XCDs in
// contiguous runs.  With a queue (PQ true, the persistent form: fewer
// workgroups than tiles) the tiles are split into the same 8 contiguous runs,
// and each workgroup takes the next tile of run blockIdx.x % 8 from the counter
// queue[8 k + run] (an atomic add) until the run is used up; no workgroup waits
// for another, and every one stops once its counter passes the run's end.  A
// tile's results do not depend on which workgroup computes it.  The two forms
// are separate kernels: the loop raises the register count of the transposed
// step (161 to 225 VGPRs at C = 3, R = 5), which would cost the one-tile form
// a wave per SIMD.
template <bool PQ, class Body>
__device__ __forceinline__ void for_batched_tiles(int* __restrict__ queue, int k, int total, Body&& body) {
    if constexpr (!PQ) {
        body(xcd_tile(blockIdx.x, gridDim.x));
    } else {
        // 16 bytes, so that the dynamic LDS placed after the static variables
        // stays aligned for the 16-byte slot reads
        __shared__ __align__(16) int next[4];
        const int x = blockIdx.x % 8;
        const int per = total / 8, rem = total % 8;
        const int lo = x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
        const int n = per + (x < rem ? 1 : 0);
        const bool first = threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0;
        for (;;) {
            if (first) next[0] = atomicAdd(queue + 8 * k + x, 1);
            __syncthreads();
            const int i = next[0];
            if (i >= n) break;
            body(lo + i);
            __syncthreads();  // every thread is done with the tile (and with `next`)
        }
    }
}

// Forward step k of several images in one launch: the tiles of every job,
// jobs[j].start being the first global tile of job j.
template <int CP, int RT, bool PQ>
__global__ void __launch_bounds__(kMaxThreads)
fwd_step_batched_kernel(const StepJob* __restrict__ jobs, int njobs, int k, int C, int Rrt, int total,
                        int* __restrict__ queue) {
    extern __shared__ __align__(16) float lds[];
    const int R = RT > 0 ? RT : Rrt;
    for_batched_tiles<PQ>(queue, k, total, [&](int g) {
        const StepJob& J = jobs[find_job(jobs, njobs, g)];
        const size_t f = (size_t)J.H * J.W * C;
        const float* e = J.eps + 2 * k;
        const int tile = g - J.start, trow = tile / J.tiles_x;
        fwd_tile<CP, RT>(J.traj + (size_t)k * f, J.traj + (size_t)(k + 1) * f, 0.5f * e[0], 0.5f * e[1], J.H, J.W, C,
                         R, tile - trow * J.tiles_x, trow, J.dts, J.dx2, J.dy2, lds);
    });
}

// ----------------------------------------------------------------------------
// Adjoint step.  With q = (phi'/20)(D . dp), dp = p_j - p_i:
//   acc += phi dp,  accq += q D   (the step adds acc + 20 eps_c accq),
//   sx  += d^2 q,  sc += |D|^2 q.
// The control gradient uses the symmetric-window identity
//   sum_i sum_j phi' w (p_i . D_ij) = -1/2 sum_i sum_j phi' w (D_ij . (p_j - p_i))
// (w symmetric, D antisymmetric), so dl/deps_x^k = -5 dt s sum sx and
// dl/deps_c^k = -5 dt s sum sc.  The integrands d^2 q and |D|^2 q of a pair are
// the same numbers for (i, j) and (j, i) (D and dp only change sign), so with a
// compile-time radius each pixel sums them over the forward half of its window
// (a > 0, or a = 0 and b > 0) and the workgroup doubles its sums.  Each pixel
// sums its window in FP32; the sum over pixels is carried in FP64 (the
// solver's projected steps can reach 1e13 or more, which amplifies rounding
// in this sum directly into the controls).
template <int CP, int RT, int NP, bool BORDER, int PART>
__device__ __forceinline__ void adj_window(const float* mc, const float* mp, int LW, int R,
                                           const float (&ci)[NP][CP], const float (&pi)[NP][CP],
                                           float (&acc)[NP][CP], float (&accq)[NP][CP], float (&sx)[NP],
                                           float (&sc)[NP], float Ax, float Ay, float ech, float dx2, float dy2) {
    constexpr int CS = Slot<CP>::CS;
    const int RR = RT > 0 ? RT : R;
    // r: row of the neighbour relative to the thread's first pixel; pixel m sees it at a = r - m.
    // PART 1 / 2 take the first / second half of those rows (the window split over two threads).
    const int rmid = -RR + (2 * RR + NP) / 2;
    const int rlo = PART == 2 ? rmid : -RR, rhi = PART == 1 ? rmid - 1 : RR + NP - 1;
#pragma unroll
    for (int r = rlo; r <= rhi; ++r) {
        const float* rowc = mc + r * LW * CS;
        const float* rowp = mp + r * LW * CS;
#pragma unroll
        for (int b = -RR; b <= RR; ++b) {
            float cj[CP], pj[CP], mj, unused;
            load_px<CP>(rowc + b * CS, cj, mj);
            load_px<CP>(rowp + b * CS, pj, unused);
#pragma unroll
            for (int m = 0; m < NP; ++m) {
                const int a = r - m;
                if (a < -RR || a > RR || (a == 0 && b == 0)) continue;
                const float om = fmaf(-Ax, (float)(b * b), fmaf(-Ay, (float)(a * a), 1.0f));
                const float d2 = fmaf(dx2, (float)(b * b), dy2 * (float)(a * a));
                float d[CP];
                float n2 = 0.0f;
#pragma unroll
                for (int ch = 0; ch < CP; ++ch) {
                    d[ch] = cj[ch] - ci[m][ch];
                    n2 = fmaf(d[ch], d[ch], n2);
                }
                const float t = clamp01(fmaf(-ech, n2, om));
                // phi'/20 = t^3 (t - 1), with t - 1 exact inside the fused operation;
                // phi = t^4 (5 - 4t) = t^3 + t^3 (t - 1)(1 - 4t) reuses it instead of forming t^4
                const float t3 = (t * t) * t;
                float u = fmaf(t3, t, -t3);
                float w = fmaf(u, fmaf(-4.0f, t, 1.0f), t3);
                if (BORDER) {
                    w *= mj;
                    u *= mj;
                }
                float dp[CP];
                float ddp = 0.0f;
#pragma unroll
                for (int ch = 0; ch < CP; ++ch) {
                    dp[ch] = pj[ch] - pi[m][ch];
                    ddp = fmaf(d[ch], dp[ch], ddp);
                }
                const float q = u * ddp;
#pragma unroll
                for (int ch = 0; ch < CP; ++ch) {
                    acc[m][ch] = fmaf(w, dp[ch], acc[m][ch]);
                    accq[m][ch] = fmaf(q, d[ch], accq[m][ch]);
                }
                if (RT == 0 || a > 0 || (a == 0 && b > 0)) {
                    sx[m] = fmaf(d2, q, sx[m]);
                    sc[m] = fmaf(n2, q, sc[m]);
                }
            }
        }
    }
}

// One interaction tile of a transposed step (NP pixels per thread, as in the
// forward step); part[2*tile + {0,1}], tile = trow * tiles_x + tcol (row-major),
// receives the workgroup's FP64 sums of the two control-gradient integrands.
template <int CP, int RT>
__device__ __forceinline__ void adj_tile(const float* __restrict__ c, const float* __restrict__ pin,
                                         float* __restrict__ pout, float ex, float ec, int H, int W, int C, int R,
                                         int tcol, int trow, int tiles_x, float dts, float dx2, float dy2,
                                         double* __restrict__ part, float* lds, double* red) {
    constexpr int CS = Slot<CP>::CS;
    constexpr int NP = RowsPerThread<CP>::value;
    constexpr int SPLIT = AdjSplit<CP, RT>::value;  // blockDim.z
    const int TX = blockDim.x, TY = NP * blockDim.y;
    const int x0 = tcol * TX, y0 = trow * TY;
    const int LW = TX + 2 * R, LH = TY + 2 * R;
    const bool interior = x0 >= R && y0 >= R && x0 + TX + R <= W && y0 + TY + R <= H;
    float* ldc = lds;
    float* ldp = lds + LW * LH * CS;
    stage_tile2<CP>(ldc, c, ldp, pin, H, W, C, x0, y0, R, LW, LH);
    __syncthreads();
    const int gx = x0 + threadIdx.x, gy = y0 + NP * threadIdx.y;
    const bool live = gx < W && gy < H;
    double tsx = 0.0, tsc = 0.0;
    float ci[NP][CP], pi[NP][CP], acc[NP][CP], accq[NP][CP], sx[NP], sc[NP], mi;
    if (live) {
        const float exh = 0.5f * ex, ech = 0.5f * ec;
        const int off = ((NP * threadIdx.y + R) * LW + threadIdx.x + R) * CS;
        const float* mc = ldc + off;
        const float* mp = ldp + off;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            load_px<CP>(mc + m * LW * CS, ci[m], mi);
            load_px<CP>(mp + m * LW * CS, pi[m], mi);
            sx[m] = sc[m] = 0.0f;
#pragma unroll
            for (int ch = 0; ch < CP; ++ch) acc[m][ch] = accq[m][ch] = 0.0f;
        }
        const float Ax = exh * dx2, Ay = exh * dy2;
        if constexpr (SPLIT == 1) {
            if (interior)
                adj_window<CP, RT, NP, false, 0>(mc, mp, LW, R, ci, pi, acc, accq, sx, sc, Ax, Ay, ech, dx2, dy2);
            else
                adj_window<CP, RT, NP, true, 0>(mc, mp, LW, R, ci, pi, acc, accq, sx, sc, Ax, Ay, ech, dx2, dy2);
        } else if (threadIdx.z == 0) {
            if (interior)
                adj_window<CP, RT, NP, false, 1>(mc, mp, LW, R, ci, pi, acc, accq, sx, sc, Ax, Ay, ech, dx2, dy2);
            else
                adj_window<CP, RT, NP, true, 1>(mc, mp, LW, R, ci, pi, acc, accq, sx, sc, Ax, Ay, ech, dx2, dy2);
        } else {
            if (interior)
                adj_window<CP, RT, NP, false, 2>(mc, mp, LW, R, ci, pi, acc, accq, sx, sc, Ax, Ay, ech, dx2, dy2);
            else
                adj_window<CP, RT, NP, true, 2>(mc, mp, LW, R, ci, pi, acc, accq, sx, sc, Ax, Ay, ech, dx2, dy2);
        }
    }
    if constexpr (SPLIT == 2) {
        // the second layer's sums reach the first layer's threads through LDS past the two
        // fields (quantity-major: consecutive threads, consecutive words); the first adds them,
        // so every sum is (first half of the rows) + (second half)
        constexpr int NQ = 2 * CP + 2;
        const int nt = blockDim.x * blockDim.y, tt = threadIdx.x + blockDim.x * threadIdx.y;
        float* comb = lds + 2 * LW * LH * CS;
        if (threadIdx.z == 1 && live) {
#pragma unroll
            for (int m = 0; m < NP; ++m) {
#pragma unroll
                for (int ch = 0; ch < CP; ++ch) {
                    comb[(m * NQ + ch) * nt + tt] = acc[m][ch];
                    comb[(m * NQ + CP + ch) * nt + tt] = accq[m][ch];
                }
                comb[(m * NQ + 2 * CP) * nt + tt] = sx[m];
                comb[(m * NQ + 2 * CP + 1) * nt + tt] = sc[m];
            }
        }
        __syncthreads();
        if (threadIdx.z == 0 && live) {
#pragma unroll
            for (int m = 0; m < NP; ++m) {
#pragma unroll
                for (int ch = 0; ch < CP; ++ch) {
                    acc[m][ch] += comb[(m * NQ + ch) * nt + tt];
                    accq[m][ch] += comb[(m * NQ + CP + ch) * nt + tt];
                }
                sx[m] += comb[(m * NQ + 2 * CP) * nt + tt];
                sc[m] += comb[(m * NQ + 2 * CP + 1) * nt + tt];
            }
        }
    }
    if (threadIdx.z == 0 && live) {
        const float ec20 = 20.0f * ec;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            if (gy + m >= H) break;
            float* o = pout + ((size_t)(gy + m) * W + gx) * C;
#pragma unroll
            for (int ch = 0; ch < CP; ++ch)
                if (ch < C) o[ch] = fmaf(dts, fmaf(ec20, accq[m][ch], acc[m][ch]), pi[m][ch]);
            // half-window sums count each unordered pair once
            tsx += (RT > 0 ? 2.0 : 1.0) * (double)sx[m];
            tsc += (RT > 0 ? 2.0 : 1.0) * (double)sc[m];
        }
    }
    double bx = tsx, bc = tsc;
    block_sum2_f64(bx, bc, red);
    if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) {
        const int tile = trow * tiles_x + tcol;
        part[2 * tile + 0] = bx;
        part[2 * tile + 1] = bc;
    }
}

template <int CP, int RT>
__global__ void __launch_bounds__((kMaxThreads * AdjSplit<CP, RT>::value))
__attribute__((amdgpu_waves_per_eu(AdjSplit<CP, RT>::value == 2 ? 4 : 1)))
adj_step_kernel(const float* __restrict__ c, const float* __restrict__ pin, float* __restrict__ pout,
                const float* __restrict__ eps, int k, int H, int W, int C, int Rrt, int tiles_x, int tiles_y,
                float dts, float dx2, float dy2, double* __restrict__ part) {
    extern __shared__ __align__(16) float lds[];
    __shared__ double red[16];
    const int R = RT > 0 ? RT : Rrt;
    int tcol, trow;
    if (!strip_tile(tiles_x, tiles_y, tcol, trow)) return;
    adj_tile<CP, RT>(c, pin, pout, eps[2 * k], eps[2 * k + 1], H, W, C, R, tcol, trow, tiles_x, dts, dx2, dy2, part,
                     lds, red);
}

// Transposed step k of several images in one launch.  p^{k+1} is read from
// pa when K-1-k is even, else from pb, and p^k goes to the other buffer;
// part receives K x tiles x 2 partials per job.
template <int CP, int RT, bool PQ>
__global__ void __launch_bounds__((kMaxThreads * AdjSplit<CP, RT>::value))
__attribute__((amdgpu_waves_per_eu(AdjSplit<CP, RT>::value == 2 ? 4 : 1)))
adj_step_batched_kernel(const StepJob* __restrict__ jobs, int njobs, int k, int K, int C, int Rrt, int total,
                        int* __restrict__ queue) {
    extern __shared__ __align__(16) float lds[];
    __shared__ double red[16];
    const int R = RT > 0 ? RT : Rrt;
    for_batched_tiles<PQ>(queue, k, total, [&](int g) {
        const StepJob& J = jobs[find_job(jobs, njobs, g)];
        const size_t f = (size_t)J.H * J.W * C;
        const bool even = ((K - 1 - k) & 1) == 0;
        const float* e = J.eps + 2 * k;
        const int tile = g - J.start, trow = tile / J.tiles_x;
        adj_tile<CP, RT>(J.traj + (size_t)k * f, even ? J.pa : J.pb, even ? J.pb : J.pa, e[0], e[1], J.H, J.W, C, R,
                         tile - trow * J.tiles_x, trow, J.tiles_x, J.dts, J.dx2, J.dy2,
                         J.part + (size_t)k * J.tiles * 2, lds, red);
    });
}

// ----------------------------------------------------------------------------
// Direct interaction steps, for radii past ABC_MAX_RADIUS whose tile halo leaves
// fewer than kMinTiledWaves waves per CU (or does not fit the LDS at all), up to
// the whole image: with R at least the support
// radius of eq. kernel (r_ij <= 1 needs eps_x/2 |x_j - x_i|^2 <= 1), or R
// covering the image and s = 1/N, the window sum is the un-windowed sum of
// eq. MAsystem.  These are the small images with huge windows, so the work is
// split over the window as well as over the pixels: a workgroup owns an 8 x 8
// pixel block (one pixel per lane) and S waves, and walks the block's window
// (its pixels' windows joined and clipped to the image) in image coordinates,
// wave s taking source rows r0 + s, r0 + s + S, ...  All lanes of a wave read
// the same source pixel, so its loads are wave-uniform and come through the
// scalar cache; each lane zeroes the kernel argument t of sources outside its
// own window (no test at all when the window covers the image).  Out-of-image
// neighbours never occur, and the pair (i, i) adds exact zeros.  The waves'
// sums meet in LDS and are added in wave order, so every sum has a fixed order
// whatever tile the caller asked for.  O(N (2R+1)^2) work per step.  Gradient
// partials: part[2 * block + {0, 1}], one slot per 8 x 8 block (direct_blocks).
template <int CP>
__device__ __forceinline__ void load_global_px(const float* __restrict__ p, int C, float (&v)[CP]) {
    // C == CP for 1 to 4 and 31 channels (the padded counts of those); otherwise no
    // branch: channels past C reread the last one and are replaced by 0
    constexpr bool kExact = CP <= 4 || CP == 31;
#pragma unroll
    for (int ch = 0; ch < CP; ++ch) {
        const float x = p[kExact ? ch : min(ch, C - 1)];
        v[ch] = kExact || ch < C ? x : 0.0f;
    }
}

constexpr int kDirectB = 8;

template <int CP>
struct Direct {
    static constexpr int S = CP <= 8 ? 16 : (CP <= 16 ? 8 : 4);  // waves per workgroup
};

// Adds each lane's v[0..N) over the S waves in wave order; the sums end in wave 0.
// red: S x 64 float4 of LDS.
template <int N, int S>
__device__ __forceinline__ void direct_wave_sum(float (&v)[N], float4* red) {
    const int lane = threadIdx.x, s = threadIdx.y;
#pragma unroll
    for (int q0 = 0; q0 < N; q0 += 4) {
        float x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = q0 + i < N ? v[q0 + i] : 0.0f;
        if (s > 0) red[s * kWave + lane] = make_float4(x[0], x[1], x[2], x[3]);
        __syncthreads();
        if (s == 0) {
            for (int w = 1; w < S; ++w) {
                const float4 y = red[w * kWave + lane];
                x[0] += y.x;
                x[1] += y.y;
                x[2] += y.z;
                x[3] += y.w;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (q0 + i < N) v[q0 + i] = x[i];
        }
        __syncthreads();
    }
}

template <int CP, bool MASK>
__global__ void __launch_bounds__(kWave * Direct<CP>::S)
fwd_direct_kernel(const float* __restrict__ cin, float* __restrict__ cout, const float* __restrict__ eps, int k,
                  int H, int W, int C, int R, int bw, float dts, float dx2, float dy2) {
    constexpr int S = Direct<CP>::S;
    __shared__ float4 red[S * kWave];
    // the wave index is uniform: say so, so that the window loop and its loads are scalar
    const int lane = threadIdx.x, s = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int by = blockIdx.x / bw, bx = blockIdx.x - by * bw;
    const int x0 = bx * kDirectB, y0 = by * kDirectB;
    const int gx = x0 + (lane & (kDirectB - 1)), gy = y0 + lane / kDirectB;
    const bool live = gx < W && gy < H;
    const int gxc = min(gx, W - 1), gyc = min(gy, H - 1);
    const float exh = 0.5f * eps[2 * k], ech = 0.5f * eps[2 * k + 1];
    const float Ax = exh * dx2, Ay = exh * dy2;
    const float fx = (float)gxc, fy = (float)gyc, fR = (float)R;
    float ci[CP], acc[CP];
    load_global_px<CP>(cin + ((size_t)gyc * W + gxc) * C, C, ci);
#pragma unroll
    for (int ch = 0; ch < CP; ++ch) acc[ch] = 0.0f;
    const int r0 = max(y0 - R, 0), r1 = min(y0 + kDirectB - 1 + R, H - 1);
    const int q0 = max(x0 - R, 0), q1 = min(x0 + kDirectB - 1 + R, W - 1);
    for (int jr = r0 + s; jr <= r1; jr += S) {
        const float a = (float)jr - fy;
        const float oma = fmaf(-Ay, a * a, 1.0f);
        const bool rin = !MASK || fabsf(a) <= fR;
        const float* row = cin + (size_t)jr * W * C;
#pragma unroll 4
        for (int jc = q0; jc <= q1; ++jc) {
            float cj[CP], d[CP];
            load_global_px<CP>(row + (size_t)jc * C, C, cj);
            const float b = (float)jc - fx;
            float n2 = 0.0f;
#pragma unroll
            for (int ch = 0; ch < CP; ++ch) {
                d[ch] = cj[ch] - ci[ch];
                n2 = fmaf(d[ch], d[ch], n2);
            }
            float t = clamp01(fmaf(-ech, n2, fmaf(-Ax, b * b, oma)));
            if (MASK) t = (rin && fabsf(b) <= fR) ? t : 0.0f;
            const float t2 = t * t;
            const float w = fmaf(-4.0f, t, 5.0f) * (t2 * t2);
#pragma unroll
            for (int ch = 0; ch < CP; ++ch) acc[ch] = fmaf(w, d[ch], acc[ch]);
        }
    }
    direct_wave_sum<CP, S>(acc, red);
    if (s == 0 && live) {
        float* o = cout + ((size_t)gy * W + gx) * C;
#pragma unroll
        for (int ch = 0; ch < CP; ++ch)
            if (ch < C) o[ch] = fmaf(dts, acc[ch], ci[ch]);
    }
}

// Transposed step in the direct form: v holds the lane's sums of w dp (CP), of
// q D (CP) and the two control-gradient integrands over its whole window.
template <int CP, bool MASK>
__global__ void __launch_bounds__(kWave * Direct<CP>::S)
adj_direct_kernel(const float* __restrict__ c, const float* __restrict__ pin, float* __restrict__ pout,
                  const float* __restrict__ eps, int k, int H, int W, int C, int R, int bw, float dts, float dx2,
                  float dy2, double* __restrict__ part) {
    constexpr int S = Direct<CP>::S, NQ = 2 * CP + 2;
    __shared__ float4 red[S * kWave];
    // the wave index is uniform: say so, so that the window loop and its loads are scalar
    const int lane = threadIdx.x, s = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int by = blockIdx.x / bw, bx = blockIdx.x - by * bw;
    const int x0 = bx * kDirectB, y0 = by * kDirectB;
    const int gx = x0 + (lane & (kDirectB - 1)), gy = y0 + lane / kDirectB;
    const bool live = gx < W && gy < H;
    const int gxc = min(gx, W - 1), gyc = min(gy, H - 1);
    const float ex = eps[2 * k], ec = eps[2 * k + 1];
    const float exh = 0.5f * ex, ech = 0.5f * ec, ec20 = 20.0f * ec;
    const float Ax = exh * dx2, Ay = exh * dy2;
    const float fx = (float)gxc, fy = (float)gyc, fR = (float)R;
    float ci[CP], pi[CP], v[NQ];
    load_global_px<CP>(c + ((size_t)gyc * W + gxc) * C, C, ci);
    load_global_px<CP>(pin + ((size_t)gyc * W + gxc) * C, C, pi);
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = 0.0f;
    const int r0 = max(y0 - R, 0), r1 = min(y0 + kDirectB - 1 + R, H - 1);
    const int q0 = max(x0 - R, 0), q1 = min(x0 + kDirectB - 1 + R, W - 1);
    for (int jr = r0 + s; jr <= r1; jr += S) {
        const float a = (float)jr - fy;
        const float oma = fmaf(-Ay, a * a, 1.0f);
        const float d2a = dy2 * (a * a);
        const bool rin = !MASK || fabsf(a) <= fR;
        const size_t rbase = (size_t)jr * W * C;
#pragma unroll 4
        for (int jc = q0; jc <= q1; ++jc) {
            float cj[CP], pj[CP], d[CP], dp[CP];
            load_global_px<CP>(c + rbase + (size_t)jc * C, C, cj);
            load_global_px<CP>(pin + rbase + (size_t)jc * C, C, pj);
            const float b = (float)jc - fx;
            const float d2 = fmaf(dx2, b * b, d2a);
            float n2 = 0.0f;
#pragma unroll
            for (int ch = 0; ch < CP; ++ch) {
                d[ch] = cj[ch] - ci[ch];
                n2 = fmaf(d[ch], d[ch], n2);
            }
            float t = clamp01(fmaf(-ech, n2, fmaf(-Ax, b * b, oma)));
            if (MASK) t = (rin && fabsf(b) <= fR) ? t : 0.0f;
            const float t3 = (t * t) * t;
            const float u = fmaf(t3, t, -t3);
            const float w = fmaf(u, fmaf(-4.0f, t, 1.0f), t3);
            float ddp = 0.0f;
#pragma unroll
            for (int ch = 0; ch < CP; ++ch) {
                dp[ch] = pj[ch] - pi[ch];
                ddp = fmaf(d[ch], dp[ch], ddp);
            }
            const float q = u * ddp;
#pragma unroll
            for (int ch = 0; ch < CP; ++ch) {
                v[ch] = fmaf(w, dp[ch], v[ch]);
                v[CP + ch] = fmaf(q, d[ch], v[CP + ch]);
            }
            v[2 * CP] = fmaf(d2, q, v[2 * CP]);
            v[2 * CP + 1] = fmaf(n2, q, v[2 * CP + 1]);
        }
    }
    direct_wave_sum<NQ, S>(v, red);
    if (s != 0) return;
    if (live) {
        float* o = pout + ((size_t)gy * W + gx) * C;
#pragma unroll
        for (int ch = 0; ch < CP; ++ch)
            if (ch < C) o[ch] = fmaf(dts, fmaf(ec20, v[CP + ch], v[ch]), pi[ch]);
    }
    const double bsx = wave_sum_f64(live ? (double)v[2 * CP] : 0.0);
    const double bsc = wave_sum_f64(live ? (double)v[2 * CP + 1] : 0.0);
    if (lane == 0) {
        part[2 * (size_t)blockIdx.x + 0] = bsx;
        part[2 * (size_t)blockIdx.x + 1] = bsc;
    }
}

// ----------------------------------------------------------------------------
// Wide pixels (16 to 64 channels) with a radius of 1 to 3: G = CP/8 lanes per
// pixel, each lane owning 8 channels.  A pixel slot of 31 floats per field
// would let only a few waves share a CU's LDS and keep each lane busy with
// long per-channel chains; split over lanes, a 1024-thread workgroup covers
// a 16 x 16 tile with 16 waves.  Per neighbour every lane forms its partial
// |D|^2 (and D . dp), the G lanes of the pixel add them with DPP moves
// (adjacent lanes, no LDS), all of them evaluate the kernel weight, and each
// lane updates its own 8 channels.  The tile is staged as G channel planes of
// 32-byte slots; plane g starts wide_shift(G, g) vectors into its region so
// that the G x (16/G) lanes of every 16-lane read group hit distinct banks.
// The order of every sum is fixed (channels within a lane, then the lane
// pairs, then the window in the a, b order), so results do not depend on the
// tile shape or on timing.
constexpr int kMaxWideThreads = 1024;

template <int CP>
struct Wide {
    static constexpr int G = (CP + 7) / 8;
};

__host__ __device__ constexpr int wide_shift(int G, int g) {
    return G == 2 ? g : (G == 4 ? (g & 1) + 8 * (g >> 1) : (g & 1) + 4 * (g >> 1));
}

// Floats per channel plane: 32-byte slots, rounded to 256 bytes, plus room for the shift.
__host__ __device__ constexpr int wide_plane_floats(int LW, int LH) {
    return ((LW * LH * 32 + 255) / 256 * 256 + 256) / 4;
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over the G adjacent lanes of a pixel; every lane gets the same bits.
template <int G>
__device__ __forceinline__ float group_sum(float x) {
    x = x + dpp_mov<0xB1>(x);                         // quad_perm [1,0,3,2]
    if constexpr (G >= 4) x = x + dpp_mov<0x4E>(x);  // quad_perm [2,3,0,1]
    if constexpr (G >= 8) x = x + dpp_mov<0x141>(x); // row_half_mirror
    return x;
}

__device__ __forceinline__ void load8(const float* p, float (&v)[8]) {
    const float4 a = reinterpret_cast<const float4*>(p)[0];
    const float4 b = reinterpret_cast<const float4*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

// Stage rows [y0-R, y0+TY+R) x cols [x0-R, x0+TX+R) of an HWC field as G
// channel planes: thread (x, y) of the (TX G) x TY workgroup fills plane
// x % G of cell x / G in every TY-th row, 8 channels as two 16-byte vectors
// (the G lanes of a cell read one contiguous run of 4C bytes).  Cells
// outside the image and channels >= C are 0.  Every lane loads its 8
// channels without branches: a lane whose channels run past C reads on into
// the next pixel (only the image's last pixel takes clamped offsets, so no
// read leaves the field), cells outside the image read pixel 0, and the
// unwanted values are replaced by 0 afterwards.  Each row pass has the loads
// of two cells in flight before it writes LDS.
template <int G>
__device__ __forceinline__ void stage_wide(float* dst, const float* __restrict__ src, int H, int W, int C, int x0,
                                           int y0, int R, int LW, int LH, int pf) {
    const int nx = LW * G;
    const int g = threadIdx.x % G;  // blockDim.x is a multiple of G
    const int c0 = min(8 * g, C - 1);
    const int nvalid = min(8, C - 8 * g);
    const size_t last = (size_t)H * W - 1;
    for (int ly = threadIdx.y; ly < LH; ly += blockDim.y) {
        const int gy = y0 - R + ly;
        const bool row_in = (unsigned)gy < (unsigned)H;
        for (int e0 = threadIdx.x; e0 < nx; e0 += 2 * blockDim.x) {
            float v[2][8];
            int lxs[2];
            bool act[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = e0 + u * blockDim.x;
                act[u] = e < nx;
                const int lx = (act[u] ? e : 0) / G;
                lxs[u] = lx;
                const int gx = x0 - R + lx;
                const bool in = act[u] && row_in && (unsigned)gx < (unsigned)W;
                const size_t pix = in ? (size_t)gy * W + gx : 0;
                const float* p = src + pix * C + c0;
                float x[8];
                if (pix == last) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) x[k] = p[min(k, C - 1 - c0)];
                } else {
#pragma unroll
                    for (int k = 0; k < 8; ++k) x[k] = p[k];
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) v[u][k] = (in && k < nvalid) ? x[k] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (!act[u]) continue;
                float4* d = reinterpret_cast<float4*>(dst + g * pf + wide_shift(G, g) * 4 + (ly * LW + lxs[u]) * 8);
                d[0] = make_float4(v[u][0], v[u][1], v[u][2], v[u][3]);
                d[1] = make_float4(v[u][4], v[u][5], v[u][6], v[u][7]);
            }
        }
    }
}

template <int G, int RT, bool BORDER>
__device__ __forceinline__ void fwd_window_wide(const float* me, int LW, const float (&ci)[8], float (&acc)[8],
                                                float Ax, float Ay, float ech, int gx, int gy, int H, int W) {
#pragma unroll 1
    for (int a = -RT; a <= RT; ++a) {
        const float om_row = fmaf(-Ay, (float)(a * a), 1.0f);
        const bool row_in = (unsigned)(gy + a) < (unsigned)H;
#pragma unroll
        for (int b = -RT; b <= RT; ++b) {
            if (a == 0 && b == 0) continue;
            float cj[8];
            load8(me + (a * LW + b) * 8, cj);
            const float om = fmaf(-Ax, (float)(b * b), om_row);
            float d[8];
            float n2 = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                d[k] = cj[k] - ci[k];
                n2 = fmaf(d[k], d[k], n2);
            }
            n2 = group_sum<G>(n2);
            const float t = clamp01(fmaf(-ech, n2, om));
            const float t2 = t * t;
            float w = fmaf(-4.0f, t, 5.0f) * (t2 * t2);
            if (BORDER) w *= (row_in && (unsigned)(gx + b) < (unsigned)W) ? 1.0f : 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] = fmaf(w, d[k], acc[k]);
        }
    }
}

template <int CP, int RT>
__device__ __forceinline__ void fwd_tile_wide(const float* __restrict__ cin, float* __restrict__ cout, float exh,
                                              float ech, int H, int W, int C, int tcol, int trow, float dts,
                                              float dx2, float dy2, float* lds) {
    constexpr int G = Wide<CP>::G;
    const int TX = blockDim.x / G, TY = blockDim.y;
    const int x0 = tcol * TX, y0 = trow * TY;
    const int LW = TX + 2 * RT, LH = TY + 2 * RT;
    const int pf = wide_plane_floats(LW, LH);
    const bool interior = x0 >= RT && y0 >= RT && x0 + TX + RT <= W && y0 + TY + RT <= H;
    stage_wide<G>(lds, cin, H, W, C, x0, y0, RT, LW, LH, pf);
    __syncthreads();
    const int g = threadIdx.x % G, px = threadIdx.x / G;
    const int gx = x0 + px, gy = y0 + threadIdx.y;
    const float* me = lds + g * pf + wide_shift(G, g) * 4 + ((threadIdx.y + RT) * LW + px + RT) * 8;
    float ci[8], acc[8];
    load8(me, ci);
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0f;
    if (interior)
        fwd_window_wide<G, RT, false>(me, LW, ci, acc, exh * dx2, exh * dy2, ech, gx, gy, H, W);
    else
        fwd_window_wide<G, RT, true>(me, LW, ci, acc, exh * dx2, exh * dy2, ech, gx, gy, H, W);
    if (gx < W && gy < H) {
        float* o = cout + ((size_t)gy * W + gx) * C + 8 * g;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (8 * g + k < C) o[k] = fmaf(dts, acc[k], ci[k]);
    }
}

template <int G, int RT, bool BORDER>
__device__ __forceinline__ void adj_window_wide(const float* mc, const float* mp, int LW, const float (&ci)[8],
                                                const float (&pi)[8], float (&acc)[8], float& sx, float& sc, float Ax,
                                                float Ay, float ech, float ec20, float dx2, float dy2, int gx, int gy,
                                                int H, int W) {
#pragma unroll 1
    for (int a = -RT; a <= RT; ++a) {
        const float om_row = fmaf(-Ay, (float)(a * a), 1.0f);
        const float d2_row = dy2 * (float)(a * a);
        const bool row_in = (unsigned)(gy + a) < (unsigned)H;
#pragma unroll
        for (int b = -RT; b <= RT; ++b) {
            if (a == 0 && b == 0) continue;
            float cj[8], pj[8];
            load8(mc + (a * LW + b) * 8, cj);
            load8(mp + (a * LW + b) * 8, pj);
            const float om = fmaf(-Ax, (float)(b * b), om_row);
            const float d2 = fmaf(dx2, (float)(b * b), d2_row);
            float d[8], dp[8];
            float n2 = 0.0f, ddp = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                d[k] = cj[k] - ci[k];
                n2 = fmaf(d[k], d[k], n2);
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                dp[k] = pj[k] - pi[k];
                ddp = fmaf(d[k], dp[k], ddp);
            }
            n2 = group_sum<G>(n2);
            ddp = group_sum<G>(ddp);
            const float t = clamp01(fmaf(-ech, n2, om));
            const float t2 = t * t;
            const float t3 = t2 * t;
            float w = fmaf(-4.0f, t, 5.0f) * (t2 * t2);
            float u = fmaf(t3, t, -t3);  // t^3 (t - 1) in one fused operation
            if (BORDER) {
                const float m = (row_in && (unsigned)(gx + b) < (unsigned)W) ? 1.0f : 0.0f;
                w *= m;
                u *= m;
            }
            const float q = u * ddp;
            const float coef = ec20 * q;
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] = fmaf(coef, d[k], fmaf(w, dp[k], acc[k]));
            sx = fmaf(d2, q, sx);
            sc = fmaf(n2, q, sc);
        }
    }
}

template <int CP, int RT>
__device__ __forceinline__ void adj_tile_wide(const float* __restrict__ c, const float* __restrict__ pin,
                                              float* __restrict__ pout, float ex, float ec, int H, int W, int C,
                                              int tcol, int trow, int tiles_x, float dts, float dx2, float dy2,
                                              double* __restrict__ part, float* lds, double* red) {
    constexpr int G = Wide<CP>::G;
    const int TX = blockDim.x / G, TY = blockDim.y;
    const int x0 = tcol * TX, y0 = trow * TY;
    const int LW = TX + 2 * RT, LH = TY + 2 * RT;
    const int pf = wide_plane_floats(LW, LH);
    const bool interior = x0 >= RT && y0 >= RT && x0 + TX + RT <= W && y0 + TY + RT <= H;
    float* ldc = lds;
    float* ldp = lds + G * pf;
    stage_wide<G>(ldc, c, H, W, C, x0, y0, RT, LW, LH, pf);
    stage_wide<G>(ldp, pin, H, W, C, x0, y0, RT, LW, LH, pf);
    __syncthreads();
    const int g = threadIdx.x % G, px = threadIdx.x / G;
    const int gx = x0 + px, gy = y0 + threadIdx.y;
    const int off = g * pf + wide_shift(G, g) * 4 + ((threadIdx.y + RT) * LW + px + RT) * 8;
    const float* mc = ldc + off;
    const float* mp = ldp + off;
    float ci[8], pi[8], acc[8];
    load8(mc, ci);
    load8(mp, pi);
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0f;
    float sx = 0.0f, sc = 0.0f;
    const float exh = 0.5f * ex, ech = 0.5f * ec;
    if (interior)
        adj_window_wide<G, RT, false>(mc, mp, LW, ci, pi, acc, sx, sc, exh * dx2, exh * dy2, ech, 20.0f * ec, dx2,
                                      dy2, gx, gy, H, W);
    else
        adj_window_wide<G, RT, true>(mc, mp, LW, ci, pi, acc, sx, sc, exh * dx2, exh * dy2, ech, 20.0f * ec, dx2,
                                     dy2, gx, gy, H, W);
    const bool valid = gx < W && gy < H;
    if (valid) {
        float* o = pout + ((size_t)gy * W + gx) * C + 8 * g;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (8 * g + k < C) o[k] = fmaf(dts, acc[k], pi[k]);
    }
    // every lane of a pixel holds the same integrands; lane 0 contributes them
    if (!valid || g != 0) sx = sc = 0.0f;
    const double bx = block_sum_f64((double)sx, red);
    const double bc = block_sum_f64((double)sc, red);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        const int tile = trow * tiles_x + tcol;
        part[2 * tile + 0] = bx;
        part[2 * tile + 1] = bc;
    }
}

template <int CP, int RT>
__global__ void __launch_bounds__(kMaxWideThreads)
fwd_step_wide_kernel(const float* __restrict__ cin, float* __restrict__ cout, const float* __restrict__ eps, int k,
                     int H, int W, int C, int tiles_x, int tiles_y, float dts, float dx2, float dy2) {
    extern __shared__ __align__(16) float lds[];
    int tcol, trow;
    if (!strip_tile(tiles_x, tiles_y, tcol, trow)) return;
    fwd_tile_wide<CP, RT>(cin, cout, 0.5f * eps[2 * k], 0.5f * eps[2 * k + 1], H, W, C, tcol, trow, dts, dx2, dy2,
                          lds);
}

template <int CP, int RT, bool PQ>
__global__ void __launch_bounds__(kMaxWideThreads)
fwd_step_batched_wide_kernel(const StepJob* __restrict__ jobs, int njobs, int k, int C, int total,
                             int* __restrict__ queue) {
    extern __shared__ __align__(16) float lds[];
    for_batched_tiles<PQ>(queue, k, total, [&](int g) {
        const StepJob& J = jobs[find_job(jobs, njobs, g)];
        const size_t f = (size_t)J.H * J.W * C;
        const float* e = J.eps + 2 * k;
        const int tile = g - J.start, trow = tile / J.tiles_x;
        fwd_tile_wide<CP, RT>(J.traj + (size_t)k * f, J.traj + (size_t)(k + 1) * f, 0.5f * e[0], 0.5f * e[1], J.H,
                              J.W, C, tile - trow * J.tiles_x, trow, J.dts, J.dx2, J.dy2, lds);
    });
}

template <int CP, int RT>
__global__ void __launch_bounds__(kMaxWideThreads)
adj_step_wide_kernel(const float* __restrict__ c, const float* __restrict__ pin, float* __restrict__ pout,
                     const float* __restrict__ eps, int k, int H, int W, int C, int tiles_x, int tiles_y, float dts,
                     float dx2, float dy2, double* __restrict__ part) {
    extern __shared__ __align__(16) float lds[];
    __shared__ double red[16];
    int tcol, trow;
    if (!strip_tile(tiles_x, tiles_y, tcol, trow)) return;
    adj_tile_wide<CP, RT>(c, pin, pout, eps[2 * k], eps[2 * k + 1], H, W, C, tcol, trow, tiles_x, dts, dx2, dy2,
                          part, lds, red);
}

template <int CP, int RT, bool PQ>
__global__ void __launch_bounds__(kMaxWideThreads)
adj_step_batched_wide_kernel(const StepJob* __restrict__ jobs, int njobs, int k, int K, int C, int total,
                             int* __restrict__ queue) {
    extern __shared__ __align__(16) float lds[];
    __shared__ double red[16];
    for_batched_tiles<PQ>(queue, k, total, [&](int g) {
        const StepJob& J = jobs[find_job(jobs, njobs, g)];
        const size_t f = (size_t)J.H * J.W * C;
        const bool even = ((K - 1 - k) & 1) == 0;
        const float* e = J.eps + 2 * k;
        const int tile = g - J.start, trow = tile / J.tiles_x;
        adj_tile_wide<CP, RT>(J.traj + (size_t)k * f, even ? J.pa : J.pb, even ? J.pb : J.pa, e[0], e[1], J.H, J.W,
                              C, tile - trow * J.tiles_x, trow, J.tiles_x, J.dts, J.dx2, J.dy2,
                              J.part + (size_t)k * J.tiles * 2, lds, red);
    });
}

// ----------------------------------------------------------------------------
// Reductions over workgroup partials: grid (nrows, nq); each workgroup sums one
// column of one row with strided per-thread sums followed by the block tree.
__global__ void __launch_bounds__(kMaxThreads)
reduce_rows_kernel(const float* __restrict__ part, int nblk, int nq, float scale, float* __restrict__ out) {
    __shared__ float red[16];
    const int r = blockIdx.x, q = blockIdx.y;
    const float* base = part + (size_t)r * nblk * nq + q;
    float s = 0.0f;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += base[(size_t)i * nq];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[r * nq + q] = scale * s;
}

// FP64 variant for the control-gradient partials; writes FP64 and, when
// out_f is set, an FP32 copy.
__global__ void __launch_bounds__(kMaxThreads)
reduce_rows_f64_kernel(const double* __restrict__ part, int nblk, int nq, double scale, double* __restrict__ out,
                       float* __restrict__ out_f) {
    __shared__ double red[16];
    const int r = blockIdx.x, q = blockIdx.y;
    const double* base = part + (size_t)r * nblk * nq + q;
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += base[(size_t)i * nq];
    s = block_sum_f64(s, red);
    if (threadIdx.x == 0) {
        if (out) out[r * nq + q] = scale * s;
        if (out_f) out_f[r * nq + q] = (float)(scale * s);
    }
}

// Per-job reductions of FP64 rows (grid: rows x jobs x nq) and FP32 rows
// (grid: jobs x nq), each with the same per-thread strides and block tree as
// the single-image kernels above, so that a job's sums equal the single-image
// ones bit for bit.
__global__ void __launch_bounds__(kMaxThreads)
reduce_jobs_f64_kernel(const RedJob* __restrict__ jobs, int nq) {
    __shared__ double red[16];
    const RedJob& J = jobs[blockIdx.y];
    const int r = blockIdx.x, q = blockIdx.z;
    if (r >= J.rows) return;
    const double* base = J.part_d + (size_t)r * J.nblk * nq + q;
    double s = 0.0;
    for (int i = threadIdx.x; i < J.nblk; i += blockDim.x) s += base[(size_t)i * nq];
    s = block_sum_f64(s, red);
    if (threadIdx.x == 0) J.out_d[r * nq + q] = J.scale * s;
}

__global__ void __launch_bounds__(kMaxThreads)
reduce_jobs_kernel(const RedJob* __restrict__ jobs, int nq) {
    __shared__ float red[16];
    const RedJob& J = jobs[blockIdx.x];
    const int q = blockIdx.y;
    const float* base = J.part_f + q;
    float s = 0.0f;
    for (int i = threadIdx.x; i < J.nblk; i += blockDim.x) s += base[(size_t)i * nq];
    s = block_sum(s, red);
    if (threadIdx.x == 0) J.out_f[q] = s;
}

// ----------------------------------------------------------------------------
// Per-pixel primal/dual kernels.  grad# is the central difference of Def. 3.1,
// zero on the first/last column (row) by the reflective rule.  One workgroup
// covers 256 consecutive pixels (a contiguous range of every HWC field); the
// ranges are handed to the XCDs in contiguous runs, so the rows above and
// below a range are mostly in the same L2.  CP is the padded channel count:
// the channel loops unroll and every load of a pixel is in flight at once.

// Centred differences of grad# (Def. 3.1), 0 where the stencil leaves the image.
// The loads are unconditional: where the difference does not exist both indices
// are i, and x - x = +0 gives the 0 bit for bit for finite fields.
__device__ __forceinline__ float grad_x(const float* __restrict__ c, size_t i, int q, int W, int C, int ch,
                                        float inv2dx) {
    const bool ok = q >= 1 && q <= W - 2;
    const size_t a = ok ? i + 1 : i, b = ok ? i - 1 : i;
    return (c[a * C + ch] - c[b * C + ch]) * inv2dx;
}

__device__ __forceinline__ float grad_y(const float* __restrict__ c, size_t i, int r, int H, int W, int C,
                                        int ch, float inv2dy) {
    const bool ok = r >= 1 && r <= H - 2;
    const size_t a = ok ? i + (size_t)W : i, b = ok ? i - (size_t)W : i;
    return (c[a * C + ch] - c[b * C + ch]) * inv2dy;
}

// gK = area [ div(mu + rho (v - grad c)) + alpha (c - c0) ], div = -grad#^T, and the
// workgroup sums of the per-pixel objective rho/2 |v - g + mu/rho|^2 + |v| + alpha/2 |c - c0|^2,
// of |grad c| and of |c - c0|^2 (kTermQuantities values per workgroup).
// FAST: C == CP and v, mu given, so the channel loop and the loads carry no
// conditions and the scheduler can put a pixel's loads of every channel in
// flight together.
template <int CP, bool FAST>
__device__ __forceinline__ void terminal_block(const float* __restrict__ c, const float* __restrict__ c0,
                                               const float* __restrict__ v, const float* __restrict__ mu, int H, int W,
                                               int C, float rho, float alpha, float area, float inv2dx, float inv2dy,
                                               float* __restrict__ pK, float* __restrict__ part, int blk, float* red) {
    const size_t N = (size_t)H * W;
    const size_t i = (size_t)blk * blockDim.x + threadIdx.x;
    float obj = 0.0f, tv = 0.0f, fid = 0.0f;
    if (i < N) {
        const unsigned iu = (unsigned)i;  // H W C <= 4e9: pixel indices fit 32 bits
        const int r = (int)(iu / (unsigned)W), q = (int)(iu % (unsigned)W);
        const float inv_rho = 1.0f / rho;
        // gx, gy at i exist for 1 <= q <= W-2 (rows likewise); the divergence takes
        // the neighbours whose own gradient exists (xr: q+1 <= W-2, ...).  Every
        // load is unconditional, at the neighbour's index or at i where the term
        // does not exist, and a missing divergence term is multiplied by 0 (no
        // branch the compiler could sink the loads into), so the loads of a pixel
        // are in flight together.  For finite fields the results equal those of
        // skipping the term bit for bit (dv is never -0, so adding a signed zero
        // leaves it unchanged); a non-finite v, mu or c at a border pixel makes
        // its dropped term, and so its gradient entry, NaN, as its objective
        // terms already are.
        const bool gxi = q >= 1 && q <= W - 2, gyi = r >= 1 && r <= H - 2;
        const bool xl = q - 1 >= 1, xr = q + 1 <= W - 2, yu = r - 1 >= 1, yd = r + 1 <= H - 2;
        const size_t sW = (size_t)W;
        const size_t ixp = gxi ? i + 1 : i, ixm = gxi ? i - 1 : i, iyp = gyi ? i + sW : i, iym = gyi ? i - sW : i;
        const size_t jr = xr ? i + 1 : i, jl = xl ? i - 1 : i, jd = yd ? i + sW : i, ju = yu ? i - sW : i;
        const size_t jrr = xr ? i + 2 : i, jll = xl ? i - 2 : i, jdd = yd ? i + 2 * sW : i, juu = yu ? i - 2 * sW : i;
        const float mr = xr ? 1.0f : 0.0f, ml = xl ? 1.0f : 0.0f, md = yd ? 1.0f : 0.0f, mu_ = yu ? 1.0f : 0.0f;
        float sh2 = 0.0f, nv2 = 0.0f, nf2 = 0.0f, ng2 = 0.0f;
#pragma unroll
        for (int ch = 0; ch < CP; ++ch) {
            if (!FAST && ch >= C) break;
            const float cc = c[i * C + ch];
            // where the gradient does not exist both indices are i and the difference is +0
            const float gx = (c[ixp * C + ch] - c[ixm * C + ch]) * inv2dx;
            const float gy = (c[iyp * C + ch] - c[iym * C + ch]) * inv2dy;
            const float vx = (FAST || v) ? v[(i * 2 + 0) * C + ch] : 0.0f;
            const float vy = (FAST || v) ? v[(i * 2 + 1) * C + ch] : 0.0f;
            const float mx = (FAST || mu) ? mu[(i * 2 + 0) * C + ch] : 0.0f;
            const float my = (FAST || mu) ? mu[(i * 2 + 1) * C + ch] : 0.0f;
            const float shx = fmaf(mx, inv_rho, vx - gx);
            const float shy = fmaf(my, inv_rho, vy - gy);
            sh2 = fmaf(shx, shx, fmaf(shy, shy, sh2));
            nv2 = fmaf(vx, vx, fmaf(vy, vy, nv2));
            ng2 = fmaf(gx, gx, fmaf(gy, gy, ng2));
            const float e = cc - c0[i * C + ch];
            nf2 = fmaf(e, e, nf2);
        }
        // the gradient output in a loop of its own, so that a channel's loads do not
        // wait behind the previous channel's store
        if (pK) {
#pragma unroll
            for (int ch = 0; ch < CP; ++ch) {
                if (!FAST && ch >= C) break;
                const float cc = c[i * C + ch];
                const float e = cc - c0[i * C + ch];
                float dv = 0.0f;
                {
                    const float g = (c[jrr * C + ch] - cc) * inv2dx;
                    const float vv = (FAST || v) ? v[(jr * 2 + 0) * C + ch] : 0.0f;
                    const float mm = (FAST || mu) ? mu[(jr * 2 + 0) * C + ch] : 0.0f;
                    dv = fmaf(fmaf(rho, vv - g, mm) * mr, inv2dx, dv);
                }
                {
                    const float g = (cc - c[jll * C + ch]) * inv2dx;
                    const float vv = (FAST || v) ? v[(jl * 2 + 0) * C + ch] : 0.0f;
                    const float mm = (FAST || mu) ? mu[(jl * 2 + 0) * C + ch] : 0.0f;
                    dv = fmaf(-fmaf(rho, vv - g, mm) * ml, inv2dx, dv);
                }
                {
                    const float g = (c[jdd * C + ch] - cc) * inv2dy;
                    const float vv = (FAST || v) ? v[(jd * 2 + 1) * C + ch] : 0.0f;
                    const float mm = (FAST || mu) ? mu[(jd * 2 + 1) * C + ch] : 0.0f;
                    dv = fmaf(fmaf(rho, vv - g, mm) * md, inv2dy, dv);
                }
                {
                    const float g = (cc - c[juu * C + ch]) * inv2dy;
                    const float vv = (FAST || v) ? v[(ju * 2 + 1) * C + ch] : 0.0f;
                    const float mm = (FAST || mu) ? mu[(ju * 2 + 1) * C + ch] : 0.0f;
                    dv = fmaf(-fmaf(rho, vv - g, mm) * mu_, inv2dy, dv);
                }
                pK[i * C + ch] = area * fmaf(alpha, e, dv);
            }
        }
        obj = fmaf(0.5f * rho, sh2, sqrtf(nv2)) + 0.5f * alpha * nf2;
        tv = sqrtf(ng2);
        fid = nf2;
    }
    obj = block_sum(obj, red);
    tv = block_sum(tv, red);
    fid = block_sum(fid, red);
    if (threadIdx.x == 0) {
        part[(size_t)blk * kTermQuantities + 0] = obj;
        part[(size_t)blk * kTermQuantities + 1] = tv;
        part[(size_t)blk * kTermQuantities + 2] = fid;
    }
}

template <int CP>
__global__ void __launch_bounds__(kMaxThreads)
terminal_kernel(const float* __restrict__ c, const float* __restrict__ c0, const float* __restrict__ v,
                const float* __restrict__ mu, int H, int W, int C, float rho, float alpha, float area,
                float inv2dx, float inv2dy, float* __restrict__ pK, float* __restrict__ part) {
    __shared__ float red[16];
    if (C == CP && v && mu)
        terminal_block<CP, true>(c, c0, v, mu, H, W, CP, rho, alpha, area, inv2dx, inv2dy, pK, part,
                                 xcd_tile(blockIdx.x, gridDim.x), red);
    else
        terminal_block<CP, false>(c, c0, v, mu, H, W, C, rho, alpha, area, inv2dx, inv2dy, pK, part,
                                  xcd_tile(blockIdx.x, gridDim.x), red);
}

// Terminal condition / objective of several images: jobs[j].start is the first
// global block of job j (one block = 256 consecutive pixels of one image).
template <int CP>
__global__ void __launch_bounds__(kMaxThreads)
terminal_batched_kernel(const PixJob* __restrict__ jobs, int njobs, int C, float rho, float alpha) {
    __shared__ float red[16];
    const int g = xcd_tile(blockIdx.x, gridDim.x);
    const PixJob& J = jobs[find_job(jobs, njobs, g)];
    if (C == CP && J.v && J.mu)
        terminal_block<CP, true>(J.c, J.c0, J.v, J.mu, J.H, J.W, CP, rho, alpha, J.area, J.inv2dx, J.inv2dy, J.pK,
                                 J.part, g - J.start, red);
    else
        terminal_block<CP, false>(J.c, J.c0, J.v, J.mu, J.H, J.W, C, rho, alpha, J.area, J.inv2dx, J.inv2dy, J.pK,
                                  J.part, g - J.start, red);
}

// v = shrink(grad c - mu/rho) jointly over the 2C components of each pixel;
// mu += gamma (v - grad c) when update_mu.  Partial sums (kPdQuantities).
// Two passes over the workgroup's pixel range: one thread per pixel finds the
// shrink factor and the per-pixel norms, then one thread per v/mu entry
// (consecutive threads on consecutive floats) writes v and mu.  EXACT: C == CP,
// so the channel loop has no conditions and 2C is a constant.
template <int CP, bool EXACT>
__device__ __forceinline__ void pd_block(const float* __restrict__ c, const float* __restrict__ c0,
                                         float* __restrict__ v, float* __restrict__ mu, int update_mu, int H, int W,
                                         int C, float rho, float gamma, float inv2dx, float inv2dy,
                                         float* __restrict__ part, int blk, float* red, float* fac_s) {
    const size_t N = (size_t)H * W;
    const size_t p0 = (size_t)blk * blockDim.x;
    const size_t i = p0 + threadIdx.x;
    const float inv_rho = 1.0f / rho;
    float qv[kPdQuantities] = {0, 0, 0, 0, 0, 0, 0};
    if (i < N) {
        const unsigned iu = (unsigned)i;  // H W C <= 4e9: pixel indices fit 32 bits
        const int r = (int)(iu / (unsigned)W), q = (int)(iu % (unsigned)W);
        float na2 = 0.0f, ng2 = 0.0f, sf = 0.0f;
#pragma unroll
        for (int ch = 0; ch < CP; ++ch) {
            if (!EXACT && ch >= C) break;
            const float gx = grad_x(c, i, q, W, C, ch, inv2dx);
            const float gy = grad_y(c, i, r, H, W, C, ch, inv2dy);
            const float ax = gx - mu[(i * 2 + 0) * C + ch] * inv_rho;
            const float ay = gy - mu[(i * 2 + 1) * C + ch] * inv_rho;
            na2 = fmaf(ax, ax, fmaf(ay, ay, na2));
            ng2 = fmaf(gx, gx, fmaf(gy, gy, ng2));
            const float e = c[i * C + ch] - c0[i * C + ch];
            sf = fmaf(e, e, sf);
        }
        const float na = sqrtf(na2);
        const float fac = na > inv_rho ? (na - inv_rho) / na : 0.0f;
        fac_s[threadIdx.x] = fac;
        const float nv = fac * na;  // |v| of the pixel
        qv[1] = ng2;
        qv[2] = nv * nv;
        qv[3] = sqrtf(ng2);
        qv[4] = sf;
        qv[5] = nv;
        qv[6] = nv;
    }
    __syncthreads();
    // Entries are indexed from the workgroup's first pixel p0 (32-bit: at most
    // blockDim.x * 2C of them); row and column come from p0's in 32-bit division.
    const unsigned n2c = 2u * (unsigned)C;
    const size_t pend = p0 + blockDim.x < N ? p0 + blockDim.x : N;
    const unsigned nloc = (unsigned)(pend > p0 ? pend - p0 : 0) * n2c;
    const unsigned p0u = (unsigned)p0;  // H W C <= 4e9: pixel indices fit 32 bits
    const unsigned r0 = p0u / (unsigned)W, q0 = p0u % (unsigned)W;
    float svg = 0.0f, muvg = 0.0f, sh2 = 0.0f;
    // two entries per pass (el and el + blockDim.x), loaded together; the sums
    // take them in the order of a one-entry loop
    for (unsigned el0 = threadIdx.x; el0 < nloc; el0 += 2 * blockDim.x) {
        float g[2], m[2];
        size_t e[2];
        unsigned lps[2];
        bool act[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            act[u] = el0 + u * blockDim.x < nloc;
            const unsigned el = act[u] ? el0 + u * blockDim.x : el0;  // a spare lane reloads el0
            const unsigned lp = el / n2c;
            const int rem = (int)(el - lp * n2c);
            const int dim = rem >= C;
            const int ch = rem - dim * C;
            const size_t px = p0 + lp;
            const unsigned qq = q0 + lp;
            const int r = (int)(r0 + qq / (unsigned)W), q = (int)(qq % (unsigned)W);
            e[u] = p0 * (size_t)n2c + el;
            // grad_x or grad_y of the entry without a branch (dim differs between lanes)
            const bool ok = dim == 0 ? (q >= 1 && q <= W - 2) : (r >= 1 && r <= H - 2);
            const size_t step = dim == 0 ? 1 : (size_t)W;
            const size_t ia = ok ? px + step : px, ib = ok ? px - step : px;
            g[u] = (c[ia * C + ch] - c[ib * C + ch]) * (dim == 0 ? inv2dx : inv2dy);
            m[u] = mu[e[u]];
            lps[u] = lp;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (!act[u]) break;
            const float vn = fac_s[lps[u]] * (g[u] - m[u] * inv_rho);
            const float mn = update_mu ? fmaf(gamma, vn - g[u], m[u]) : m[u];
            v[e[u]] = vn;
            if (update_mu) mu[e[u]] = mn;
            const float vg = vn - g[u];
            svg = fmaf(vg, vg, svg);
            muvg = fmaf(mn, vg, muvg);
            const float sh = fmaf(mn, inv_rho, vg);
            sh2 = fmaf(sh, sh, sh2);
        }
    }
    qv[0] = svg;
    qv[5] += muvg;
    qv[6] = fmaf(0.5f * rho, sh2, qv[6]);
#pragma unroll
    for (int m = 0; m < kPdQuantities; ++m) {
        const float s = block_sum(qv[m], red);
        if (threadIdx.x == 0) part[(size_t)blk * kPdQuantities + m] = s;
    }
}

template <int CP>
__global__ void __launch_bounds__(kMaxThreads)
pd_step_kernel(const float* __restrict__ c, const float* __restrict__ c0, float* __restrict__ v,
               float* __restrict__ mu, int update_mu, int H, int W, int C, float rho, float gamma,
               float inv2dx, float inv2dy, float* __restrict__ part) {
    __shared__ float red[16];
    __shared__ float fac_s[kMaxThreads];
    if (C == CP)
        pd_block<CP, true>(c, c0, v, mu, update_mu, H, W, CP, rho, gamma, inv2dx, inv2dy, part,
                           xcd_tile(blockIdx.x, gridDim.x), red, fac_s);
    else
        pd_block<CP, false>(c, c0, v, mu, update_mu, H, W, C, rho, gamma, inv2dx, inv2dy, part,
                            xcd_tile(blockIdx.x, gridDim.x), red, fac_s);
}

template <int CP>
__global__ void __launch_bounds__(kMaxThreads)
pd_step_batched_kernel(const PixJob* __restrict__ jobs, int njobs, int update_mu, int C, float rho, float gamma) {
    __shared__ float red[16];
    __shared__ float fac_s[kMaxThreads];
    const int g = xcd_tile(blockIdx.x, gridDim.x);
    const PixJob& J = jobs[find_job(jobs, njobs, g)];
    if (C == CP)
        pd_block<CP, true>(J.c, J.c0, J.v, J.mu, update_mu, J.H, J.W, CP, rho, gamma, J.inv2dx, J.inv2dy, J.part,
                           g - J.start, red, fac_s);
    else
        pd_block<CP, false>(J.c, J.c0, J.v, J.mu, update_mu, J.H, J.W, C, rho, gamma, J.inv2dx, J.inv2dy, J.part,
                            g - J.start, red, fac_s);
}

__global__ void __launch_bounds__(kMaxThreads)
nonfinite_kernel(const float* __restrict__ x, size_t n, int* __restrict__ flag) {
    int bad = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        bad |= !isfinite(x[i]);
    if (__any(bad) && (threadIdx.x % kWave) == 0) atomicOr(flag, 1);
}

// ----------------------------------------------------------------------------
// Dispatch over the padded channel count CP and the compile-time radius.
constexpr int kChannelSteps[] = {1, 2, 3, 4, 8, 16, 31, 32, 64};

int padded_channels(int C) {
    for (int cp : kChannelSteps)
        if (C <= cp) return cp;
    return -1;
}

// Calls fn(std::integral_constant<int, CP>{}) for the padded channel count of C.
template <class Fn>
hipError_t by_channels(int C, Fn&& fn) {
    switch (padded_channels(C)) {
        case 1: return fn(std::integral_constant<int, 1>{});
        case 2: return fn(std::integral_constant<int, 2>{});
        case 3: return fn(std::integral_constant<int, 3>{});
        case 4: return fn(std::integral_constant<int, 4>{});
        case 8: return fn(std::integral_constant<int, 8>{});
        case 16: return fn(std::integral_constant<int, 16>{});
        case 31: return fn(std::integral_constant<int, 31>{});
        case 32: return fn(std::integral_constant<int, 32>{});
        case 64: return fn(std::integral_constant<int, 64>{});
        default: return hipErrorInvalidValue;
    }
}

// Grid of a one-image interaction launch, in the layout strip_tile decodes.
bool strip_grid(int tiles_x, int tiles_y, dim3& grid) {
    const long bh = (tiles_y + 7) / 8, strips = (tiles_x + kStrip - 1) / kStrip;
    if (64 * bh > INT_MAX || strips > 65535) return false;
    grid = dim3((unsigned)(64 * bh), (unsigned)strips);
    return true;
}

template <int CP, int RT>
hipError_t fwd_launch_t(const float* cin, float* cout, const float* eps, int k, int H, int W, int C, int R,
                        float dts, Tile t, hipStream_t s) {
    const int tiles_x = (W + t.tx - 1) / t.tx, tiles_y = (H + t.ty - 1) / t.ty;
    dim3 grid;
    if (!strip_grid(tiles_x, tiles_y, grid)) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes(CP, R, t, 1);
    auto fn = fwd_step_kernel<CP, RT>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const float dx2 = 1.0f / ((float)W * (float)W), dy2 = 1.0f / ((float)H * (float)H);
    hipLaunchKernelGGL(fn, grid, dim3(t.tx, t.ty / RowsPerThread<CP>::value), lds, s, cin, cout, eps, k, H, W, C,
                       R, tiles_x, tiles_y, dts, dx2, dy2);
    return hipGetLastError();
}

template <int CP, int RT>
hipError_t adj_launch_t(const float* c, const float* pin, float* pout, const float* eps, int k, int H, int W,
                        int C, int R, float dts, Tile t, double* part, hipStream_t s) {
    const int tiles_x = (W + t.tx - 1) / t.tx, tiles_y = (H + t.ty - 1) / t.ty;
    dim3 grid;
    if (!strip_grid(tiles_x, tiles_y, grid)) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes(CP, R, t, 2);
    auto fn = adj_step_kernel<CP, RT>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const float dx2 = 1.0f / ((float)W * (float)W), dy2 = 1.0f / ((float)H * (float)H);
    hipLaunchKernelGGL(fn, grid, dim3(t.tx, t.ty / RowsPerThread<CP>::value, AdjSplit<CP, RT>::value), lds, s, c,
                       pin, pout, eps, k, H, W, C, R, tiles_x, tiles_y, dts, dx2, dy2, part);
    return hipGetLastError();
}

template <int CP, int RT>
hipError_t fwd_wide_launch(const float* cin, float* cout, const float* eps, int k, int H, int W, int C, float dts,
                           Tile t, hipStream_t s) {
    constexpr int G = Wide<CP>::G;
    const int tiles_x = (W + t.tx - 1) / t.tx, tiles_y = (H + t.ty - 1) / t.ty;
    dim3 grid;
    if (!strip_grid(tiles_x, tiles_y, grid)) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes(C, RT, t, 1);
    auto fn = fwd_step_wide_kernel<CP, RT>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const float dx2 = 1.0f / ((float)W * (float)W), dy2 = 1.0f / ((float)H * (float)H);
    hipLaunchKernelGGL(fn, grid, dim3(t.tx * G, t.ty), lds, s, cin, cout, eps, k, H, W, C, tiles_x, tiles_y, dts,
                       dx2, dy2);
    return hipGetLastError();
}

template <int CP, int RT>
hipError_t adj_wide_launch(const float* c, const float* pin, float* pout, const float* eps, int k, int H, int W,
                           int C, float dts, Tile t, double* part, hipStream_t s) {
    constexpr int G = Wide<CP>::G;
    const int tiles_x = (W + t.tx - 1) / t.tx, tiles_y = (H + t.ty - 1) / t.ty;
    dim3 grid;
    if (!strip_grid(tiles_x, tiles_y, grid)) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes(C, RT, t, 2);
    auto fn = adj_step_wide_kernel<CP, RT>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const float dx2 = 1.0f / ((float)W * (float)W), dy2 = 1.0f / ((float)H * (float)H);
    hipLaunchKernelGGL(fn, grid, dim3(t.tx * G, t.ty), lds, s, c, pin, pout, eps, k, H, W, C, tiles_x, tiles_y,
                       dts, dx2, dy2, part);
    return hipGetLastError();
}

template <int CP, int RT>
hipError_t fwdb_wide_launch(const StepJob* jobs, int njobs, int total, int k, int C, Tile t, int* queue,
                            hipStream_t s) {
    constexpr int G = Wide<CP>::G;
    const size_t lds = tile_lds_bytes(C, RT, t, 1);
    auto fn = queue ? fwd_step_batched_wide_kernel<CP, RT, true> : fwd_step_batched_wide_kernel<CP, RT, false>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int grid = queue ? persistent_grid(C, RT, t, 1, total) : total;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(t.tx * G, t.ty), lds, s, jobs, njobs, k, C, total, queue);
    return hipGetLastError();
}

template <int CP, int RT>
hipError_t adjb_wide_launch(const StepJob* jobs, int njobs, int total, int k, int K, int C, Tile t, int* queue,
                            hipStream_t s) {
    constexpr int G = Wide<CP>::G;
    const size_t lds = tile_lds_bytes(C, RT, t, 2);
    auto fn = queue ? adj_step_batched_wide_kernel<CP, RT, true> : adj_step_batched_wide_kernel<CP, RT, false>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int grid = queue ? persistent_grid(C, RT, t, 2, total) : total;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(t.tx * G, t.ty), lds, s, jobs, njobs, k, K, C, total, queue);
    return hipGetLastError();
}

// The window test is needed unless every pixel's window covers the image.
bool direct_masks(int H, int W, int R) { return R < H - 1 || R < W - 1; }

template <int CP>
hipError_t fwd_direct_launch(const float* cin, float* cout, const float* eps, int k, int H, int W, int C, int R,
                             float dts, hipStream_t s) {
    const int bw = (W + kDirectB - 1) / kDirectB;
    const float dx2 = 1.0f / ((float)W * (float)W), dy2 = 1.0f / ((float)H * (float)H);
    auto fn = direct_masks(H, W, R) ? fwd_direct_kernel<CP, true> : fwd_direct_kernel<CP, false>;
    hipLaunchKernelGGL(fn, dim3((unsigned)direct_blocks(H, W)), dim3(kWave, Direct<CP>::S), 0, s, cin, cout, eps, k,
                       H, W, C, R, bw, dts, dx2, dy2);
    return hipGetLastError();
}

template <int CP>
hipError_t adj_direct_launch(const float* c, const float* pin, float* pout, const float* eps, int k, int H, int W,
                             int C, int R, float dts, double* part, hipStream_t s) {
    const int bw = (W + kDirectB - 1) / kDirectB;
    const float dx2 = 1.0f / ((float)W * (float)W), dy2 = 1.0f / ((float)H * (float)H);
    auto fn = direct_masks(H, W, R) ? adj_direct_kernel<CP, true> : adj_direct_kernel<CP, false>;
    hipLaunchKernelGGL(fn, dim3((unsigned)direct_blocks(H, W)), dim3(kWave, Direct<CP>::S), 0, s, c, pin, pout, eps,
                       k, H, W, C, R, bw, dts, dx2, dy2, part);
    return hipGetLastError();
}

// Compile-time radii for the small-channel kernels (full unroll of the window);
// wider channel counts and other radii use the runtime-radius kernel.
template <int CP>
hipError_t fwd_launch_r(const float* cin, float* cout, const float* eps, int k, int H, int W, int C, int R,
                        float dts, Tile t, hipStream_t s) {
    if (direct_step(C, R, t, 1)) return fwd_direct_launch<CP>(cin, cout, eps, k, H, W, C, R, dts, s);
    if constexpr (CP <= 4) {
        switch (R) {
            case 1: return fwd_launch_t<CP, 1>(cin, cout, eps, k, H, W, C, R, dts, t, s);
            case 2: return fwd_launch_t<CP, 2>(cin, cout, eps, k, H, W, C, R, dts, t, s);
            case 3: return fwd_launch_t<CP, 3>(cin, cout, eps, k, H, W, C, R, dts, t, s);
            case 4: return fwd_launch_t<CP, 4>(cin, cout, eps, k, H, W, C, R, dts, t, s);
            case 5: return fwd_launch_t<CP, 5>(cin, cout, eps, k, H, W, C, R, dts, t, s);
            default: break;
        }
    } else if constexpr (CP >= 16) {
        switch (R) {
            case 1: return fwd_wide_launch<CP, 1>(cin, cout, eps, k, H, W, C, dts, t, s);
            case 2: return fwd_wide_launch<CP, 2>(cin, cout, eps, k, H, W, C, dts, t, s);
            case 3: return fwd_wide_launch<CP, 3>(cin, cout, eps, k, H, W, C, dts, t, s);
            default: break;
        }
    }
    return fwd_launch_t<CP, 0>(cin, cout, eps, k, H, W, C, R, dts, t, s);
}

template <int CP>
hipError_t adj_launch_r(const float* c, const float* pin, float* pout, const float* eps, int k, int H, int W,
                        int C, int R, float dts, Tile t, double* part, hipStream_t s) {
    if (direct_step(C, R, t, 2)) return adj_direct_launch<CP>(c, pin, pout, eps, k, H, W, C, R, dts, part, s);
    if constexpr (CP <= 4) {
        switch (R) {
            case 1: return adj_launch_t<CP, 1>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
            case 2: return adj_launch_t<CP, 2>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
            case 3: return adj_launch_t<CP, 3>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
            case 4: return adj_launch_t<CP, 4>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
            case 5: return adj_launch_t<CP, 5>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
            default: break;
        }
    } else if constexpr (CP >= 16) {
        switch (R) {
            case 1: return adj_wide_launch<CP, 1>(c, pin, pout, eps, k, H, W, C, dts, t, part, s);
            case 2: return adj_wide_launch<CP, 2>(c, pin, pout, eps, k, H, W, C, dts, t, part, s);
            case 3: return adj_wide_launch<CP, 3>(c, pin, pout, eps, k, H, W, C, dts, t, part, s);
            default: break;
        }
    }
    return adj_launch_t<CP, 0>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
}

template <int CP, int RT>
hipError_t fwdb_launch_t(const StepJob* jobs, int njobs, int total, int k, int C, int R, Tile t, int* queue,
                         hipStream_t s) {
    const size_t lds = tile_lds_bytes(CP, R, t, 1);
    auto fn = queue ? fwd_step_batched_kernel<CP, RT, true> : fwd_step_batched_kernel<CP, RT, false>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int grid = queue ? persistent_grid(C, R, t, 1, total) : total;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(t.tx, t.ty / RowsPerThread<CP>::value), lds, s, jobs, njobs, k, C, R,
                       total, queue);
    return hipGetLastError();
}

template <int CP, int RT>
hipError_t adjb_launch_t(const StepJob* jobs, int njobs, int total, int k, int K, int C, int R, Tile t, int* queue,
                         hipStream_t s) {
    const size_t lds = tile_lds_bytes(CP, R, t, 2);
    auto fn = queue ? adj_step_batched_kernel<CP, RT, true> : adj_step_batched_kernel<CP, RT, false>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int grid = queue ? persistent_grid(C, R, t, 2, total) : total;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(t.tx, t.ty / RowsPerThread<CP>::value, AdjSplit<CP, RT>::value), lds, s,
                       jobs, njobs, k, K, C, R, total, queue);
    return hipGetLastError();
}

template <int CP>
hipError_t fwdb_launch_r(const StepJob* jobs, int njobs, int total, int k, int C, int R, Tile t, int* queue,
                         hipStream_t s) {
    if constexpr (CP <= 4) {
        switch (R) {
            case 1: return fwdb_launch_t<CP, 1>(jobs, njobs, total, k, C, R, t, queue, s);
            case 2: return fwdb_launch_t<CP, 2>(jobs, njobs, total, k, C, R, t, queue, s);
            case 3: return fwdb_launch_t<CP, 3>(jobs, njobs, total, k, C, R, t, queue, s);
            case 4: return fwdb_launch_t<CP, 4>(jobs, njobs, total, k, C, R, t, queue, s);
            case 5: return fwdb_launch_t<CP, 5>(jobs, njobs, total, k, C, R, t, queue, s);
            default: break;
        }
    } else if constexpr (CP >= 16) {
        switch (R) {
            case 1: return fwdb_wide_launch<CP, 1>(jobs, njobs, total, k, C, t, queue, s);
            case 2: return fwdb_wide_launch<CP, 2>(jobs, njobs, total, k, C, t, queue, s);
            case 3: return fwdb_wide_launch<CP, 3>(jobs, njobs, total, k, C, t, queue, s);
            default: break;
        }
    }
    return fwdb_launch_t<CP, 0>(jobs, njobs, total, k, C, R, t, queue, s);
}

template <int CP>
hipError_t adjb_launch_r(const StepJob* jobs, int njobs, int total, int k, int K, int C, int R, Tile t,
                         int* queue, hipStream_t s) {
    if constexpr (CP <= 4) {
        switch (R) {
            case 1: return adjb_launch_t<CP, 1>(jobs, njobs, total, k, K, C, R, t, queue, s);
            case 2: return adjb_launch_t<CP, 2>(jobs, njobs, total, k, K, C, R, t, queue, s);
            case 3: return adjb_launch_t<CP, 3>(jobs, njobs, total, k, K, C, R, t, queue, s);
            case 4: return adjb_launch_t<CP, 4>(jobs, njobs, total, k, K, C, R, t, queue, s);
            case 5: return adjb_launch_t<CP, 5>(jobs, njobs, total, k, K, C, R, t, queue, s);
            default: break;
        }
    } else if constexpr (CP >= 16) {
        switch (R) {
            case 1: return adjb_wide_launch<CP, 1>(jobs, njobs, total, k, K, C, t, queue, s);
            case 2: return adjb_wide_launch<CP, 2>(jobs, njobs, total, k, K, C, t, queue, s);
            case 3: return adjb_wide_launch<CP, 3>(jobs, njobs, total, k, K, C, t, queue, s);
            default: break;
        }
    }
    return adjb_launch_t<CP, 0>(jobs, njobs, total, k, K, C, R, t, queue, s);
}

}  // namespace

int tile_count(int H, int W, Tile t) { return ((W + t.tx - 1) / t.tx) * ((H + t.ty - 1) / t.ty); }

// Lanes per pixel: G = CP/8 for the wide kernels (16 to 64 channels, radius 1 to 3), else 1.
int wide_lanes(int C, int R) {
    const int cp = padded_channels(C);
    return (cp >= 16 && R >= 1 && R <= 3) ? (cp + 7) / 8 : 1;
}

// Thread layers of the transposed step for (C, R) as launched (AdjSplit of the kernel that runs).
int adj_split(int C, int R) {
    const int cp = padded_channels(C);
    return cp >= 1 && cp <= 4 && R >= 1 && R <= 5 ? 2 : 1;
}

size_t tile_lds_bytes(int C, int R, Tile t, int fields) {
    const int cp = padded_channels(C);
    if (cp < 0) return (size_t)-1;
    const int G = wide_lanes(C, R);
    if (G > 1) return (size_t)fields * G * wide_plane_floats(t.tx + 2 * R, t.ty + 2 * R) * sizeof(float);
    const int nv = (cp + 1 + 3) / 4;
    const int cs = cp == 1 ? 2 : 4 * (nv % 2 ? nv : nv + 1);
    // plus the forward step's offset-constant table ((2R+1)^2 floats), and in the split
    // transposed step the second layer's sums (2 cp + 2 floats per pixel)
    const size_t comb = fields == 2 && adj_split(C, R) == 2 ? (size_t)t.tx * t.ty * (2 * cp + 2) : 0;
    return ((size_t)fields * (size_t)(t.tx + 2 * R) * (size_t)(t.ty + 2 * R) * (size_t)cs +
            (size_t)(2 * R + 1) * (2 * R + 1) + comb) * sizeof(float);
}

int rows_per_thread(int C, int R) {
    const int cp = padded_channels(C);
    if (cp < 0 || wide_lanes(C, R) > 1) return 1;
    return cp <= 4 ? RowsPerThread<4>::value : RowsPerThread<8>::value;
}

bool tile_ok(int C, int R, Tile t, int fields) {
    const int G = wide_lanes(C, R), NP = rows_per_thread(C, R);
    if (t.tx < 1 || t.ty < 1 || t.ty % NP != 0) return false;
    const int threads = t.tx * (t.ty / NP) * G;
    if (threads > (G > 1 ? kMaxWideThreads : kMaxThreads)) return false;
    if (threads % kWave != 0) return false;
    return tile_lds_bytes(C, R, t, fields) <= kMaxLds || R > ABC_MAX_RADIUS;
}


// Waves one CU can hold for a tile, limited by LDS and by 8 waves per SIMD.
static int tile_waves_per_cu(int C, int R, Tile t, int fields) {
    const int wpb = (t.tx * (t.ty / rows_per_thread(C, R)) * wide_lanes(C, R) * (fields == 2 ? adj_split(C, R) : 1) +
                     kWave - 1) / kWave;
    const size_t lds = tile_lds_bytes(C, R, t, fields);
    const int by_lds = (int)(kMaxLds / std::max<size_t>(lds, 1));
    return std::min(by_lds, 32 / wpb) * wpb;
}

// Past ABC_MAX_RADIUS a tile runs the tiled kernels only while its halo leaves
// at least this many waves per CU (measured: with 8 the tiled forward step beats
// the direct one, with 4 or fewer the direct kernels win).
constexpr int kMinTiledWaves = 8;

bool direct_step(int C, int R, Tile t, int fields) {
    return R > ABC_MAX_RADIUS && tile_waves_per_cu(C, R, t, fields) < kMinTiledWaves;
}

int direct_blocks(int H, int W) { return ((W + kDirectB - 1) / kDirectB) * ((H + kDirectB - 1) / kDirectB); }

int adj_part_count(int H, int W, int C, int R, Tile t) {
    return direct_step(C, R, t, 2) ? direct_blocks(H, W) : tile_count(H, W, t);
}

// Workgroups of a persistent multi-image launch: as many as the GPU holds at
// once for this tile (LDS and waves per SIMD), a multiple of 8, at most one per
// tile.
int persistent_grid(int C, int R, Tile t, int fields, int total) {
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
        cus[dev] = n;
    }
    const int wpb = (t.tx * (t.ty / rows_per_thread(C, R)) * wide_lanes(C, R) * (fields == 2 ? adj_split(C, R) : 1) +
                     kWave - 1) / kWave;
    const int per_cu = std::max(1, tile_waves_per_cu(C, R, t, fields) / wpb);
    const int cap = (cus[dev] * per_cu + 7) / 8 * 8;
    return std::min(total, cap);
}

// First candidate whose LDS fits in 64 KB (several workgroups per CU).  When
// that leaves fewer than 8 waves per CU (wide pixels), the candidate with the
// most waves per CU wins instead, then the one with the least halo.
Tile default_tile(int C, int R, int fields) {
    static const Tile cands[] = {{32, 16}, {32, 8}, {16, 16}, {64, 4}, {16, 8}, {32, 4}, {8, 16}, {8, 8}, {64, 2},
                                 {64, 1}};
    const size_t budget = 64 * 1024;
    for (const Tile& t : cands)
        if (tile_ok(C, R, t, fields) && tile_lds_bytes(C, R, t, fields) <= budget &&
            tile_waves_per_cu(C, R, t, fields) >= 8)
            return t;
    Tile best{0, 0};
    int best_w = 0;
    double best_eff = 0.0;
    for (const Tile& t : cands) {
        if (!tile_ok(C, R, t, fields)) continue;
        const int w = tile_waves_per_cu(C, R, t, fields);
        const double eff = (double)(t.tx * t.ty) / ((double)(t.tx + 2 * R) * (t.ty + 2 * R));
        if (w > best_w || (w == best_w && eff > best_eff)) {
            best = t;
            best_w = w;
            best_eff = eff;
        }
    }
    return best;
}

hipError_t launch_forward_step(const float* cin, float* cout, const float* eps, int k, int H, int W, int C, int R,
                               float dts, Tile t, hipStream_t s) {
    switch (padded_channels(C)) {
        case 1: return fwd_launch_r<1>(cin, cout, eps, k, H, W, C, R, dts, t, s);
        case 2: return fwd_launch_r<2>(cin, cout, eps, k, H, W, C, R, dts, t, s);
        case 3: return fwd_launch_r<3>(cin, cout, eps, k, H, W, C, R, dts, t, s);
        case 4: return fwd_launch_r<4>(cin, cout, eps, k, H, W, C, R, dts, t, s);
        case 8: return fwd_launch_r<8>(cin, cout, eps, k, H, W, C, R, dts, t, s);
        case 16: return fwd_launch_r<16>(cin, cout, eps, k, H, W, C, R, dts, t, s);
        case 31: return fwd_launch_r<31>(cin, cout, eps, k, H, W, C, R, dts, t, s);
        case 32: return fwd_launch_r<32>(cin, cout, eps, k, H, W, C, R, dts, t, s);
        case 64: return fwd_launch_r<64>(cin, cout, eps, k, H, W, C, R, dts, t, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_step(const float* c, const float* pin, float* pout, const float* eps, int k, int H,
                               int W, int C, int R, float dts, Tile t, double* part, hipStream_t s) {
    switch (padded_channels(C)) {
        case 1: return adj_launch_r<1>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
        case 2: return adj_launch_r<2>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
        case 3: return adj_launch_r<3>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
        case 4: return adj_launch_r<4>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
        case 8: return adj_launch_r<8>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
        case 16: return adj_launch_r<16>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
        case 31: return adj_launch_r<31>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
        case 32: return adj_launch_r<32>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
        case 64: return adj_launch_r<64>(c, pin, pout, eps, k, H, W, C, R, dts, t, part, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce_rows(const float* part, int nrows, int nblk, int nq, float* out, float scale,
                              hipStream_t s) {
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(nrows, nq), dim3(kMaxThreads), 0, s, part, nblk, nq, scale, out);
    return hipGetLastError();
}

hipError_t launch_reduce_rows_f64(const double* part, int nrows, int nblk, int nq, double scale, double* out,
                                  float* out_f, hipStream_t s) {
    hipLaunchKernelGGL(reduce_rows_f64_kernel, dim3(nrows, nq), dim3(kMaxThreads), 0, s, part, nblk, nq, scale, out,
                       out_f);
    return hipGetLastError();
}

hipError_t launch_forward_step_batched(const StepJob* jobs, int njobs, int total, int k, int C, int R, Tile t,
                                       int* queue, hipStream_t s) {
    switch (padded_channels(C)) {
        case 1: return fwdb_launch_r<1>(jobs, njobs, total, k, C, R, t, queue, s);
        case 2: return fwdb_launch_r<2>(jobs, njobs, total, k, C, R, t, queue, s);
        case 3: return fwdb_launch_r<3>(jobs, njobs, total, k, C, R, t, queue, s);
        case 4: return fwdb_launch_r<4>(jobs, njobs, total, k, C, R, t, queue, s);
        case 8: return fwdb_launch_r<8>(jobs, njobs, total, k, C, R, t, queue, s);
        case 16: return fwdb_launch_r<16>(jobs, njobs, total, k, C, R, t, queue, s);
        case 31: return fwdb_launch_r<31>(jobs, njobs, total, k, C, R, t, queue, s);
        case 32: return fwdb_launch_r<32>(jobs, njobs, total, k, C, R, t, queue, s);
        case 64: return fwdb_launch_r<64>(jobs, njobs, total, k, C, R, t, queue, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_step_batched(const StepJob* jobs, int njobs, int total, int k, int K, int C, int R, Tile t,
                                       int* queue, hipStream_t s) {
    switch (padded_channels(C)) {
        case 1: return adjb_launch_r<1>(jobs, njobs, total, k, K, C, R, t, queue, s);
        case 2: return adjb_launch_r<2>(jobs, njobs, total, k, K, C, R, t, queue, s);
        case 3: return adjb_launch_r<3>(jobs, njobs, total, k, K, C, R, t, queue, s);
        case 4: return adjb_launch_r<4>(jobs, njobs, total, k, K, C, R, t, queue, s);
        case 8: return adjb_launch_r<8>(jobs, njobs, total, k, K, C, R, t, queue, s);
        case 16: return adjb_launch_r<16>(jobs, njobs, total, k, K, C, R, t, queue, s);
        case 31: return adjb_launch_r<31>(jobs, njobs, total, k, K, C, R, t, queue, s);
        case 32: return adjb_launch_r<32>(jobs, njobs, total, k, K, C, R, t, queue, s);
        case 64: return adjb_launch_r<64>(jobs, njobs, total, k, K, C, R, t, queue, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_terminal_batched(const PixJob* jobs, int njobs, int total, int C, float rho, float alpha,
                                   hipStream_t s) {
    return by_channels(C, [&](auto cp) {
        hipLaunchKernelGGL(terminal_batched_kernel<decltype(cp)::value>, dim3(total), dim3(kMaxThreads), 0, s, jobs,
                           njobs, C, rho, alpha);
        return hipGetLastError();
    });
}

hipError_t launch_pd_step_batched(const PixJob* jobs, int njobs, int total, int update_mu, int C, float rho,
                                  float gamma, hipStream_t s) {
    return by_channels(C, [&](auto cp) {
        hipLaunchKernelGGL(pd_step_batched_kernel<decltype(cp)::value>, dim3(total), dim3(kMaxThreads), 0, s, jobs,
                           njobs, update_mu, C, rho, gamma);
        return hipGetLastError();
    });
}

hipError_t launch_reduce_jobs_f64(const RedJob* jobs, int njobs, int max_rows, int nq, hipStream_t s) {
    hipLaunchKernelGGL(reduce_jobs_f64_kernel, dim3(max_rows, njobs, nq), dim3(kMaxThreads), 0, s, jobs, nq);
    return hipGetLastError();
}

hipError_t launch_reduce_jobs(const RedJob* jobs, int njobs, int nq, hipStream_t s) {
    hipLaunchKernelGGL(reduce_jobs_kernel, dim3(njobs, nq), dim3(kMaxThreads), 0, s, jobs, nq);
    return hipGetLastError();
}

int pd_blocks(int H, int W) { return (int)(((size_t)H * W + kMaxThreads - 1) / kMaxThreads); }

hipError_t launch_terminal(const float* c, const float* c0, const float* v, const float* mu, int H, int W, int C,
                           float rho, float alpha, float area, float* pK, float* part, hipStream_t s) {
    const float inv2dx = 0.5f * (float)W, inv2dy = 0.5f * (float)H;
    return by_channels(C, [&](auto cp) {
        hipLaunchKernelGGL(terminal_kernel<decltype(cp)::value>, dim3(pd_blocks(H, W)), dim3(kMaxThreads), 0, s, c,
                           c0, v, mu, H, W, C, rho, alpha, area, inv2dx, inv2dy, pK, part);
        return hipGetLastError();
    });
}

hipError_t launch_pd_step(const float* c, const float* c0, float* v, float* mu, int update_mu, int H, int W, int C,
                          float rho, float gamma, float* part, hipStream_t s) {
    const float inv2dx = 0.5f * (float)W, inv2dy = 0.5f * (float)H;
    return by_channels(C, [&](auto cp) {
        hipLaunchKernelGGL(pd_step_kernel<decltype(cp)::value>, dim3(pd_blocks(H, W)), dim3(kMaxThreads), 0, s, c,
                           c0, v, mu, update_mu, H, W, C, rho, gamma, inv2dx, inv2dy, part);
        return hipGetLastError();
    });
}

hipError_t launch_nonfinite(const float* x, size_t n, int* flag, hipStream_t s) {
    const size_t want = (n + kMaxThreads - 1) / kMaxThreads;
    const int nb = (int)std::min<size_t>(std::max<size_t>(want, 1), 4096);
    hipLaunchKernelGGL(nonfinite_kernel, dim3(nb), dim3(kMaxThreads), 0, s, x, n, flag);
    return hipGetLastError();
}

}  // namespace abc
