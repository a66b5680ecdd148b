// Segment labelling and the segmentation scores of Sec. 4.4 on the GPU.
//
// The paper labels the segments of a processed image with a watershed
// (threshold 0.02) and scores the labels with the intra-region variance IRV
// (original image), the inter-region contrast IRC (processed image) and the
// validity score VS = IRV / IRC.  The watershed here is the marker-based one
// taken as a minimum spanning forest, which has a unique result and
// parallelises without a priority queue:
//
//   relief g2   |grad c|^2 with the central differences of Def. 3.1 in pixel
//               units, FP32, fixed operation order (so that every comparison
//               below is reproducible bit for bit);
//   markers     4-connected components of {g2 < theta^2}; if empty, the pixel
//               of smallest g2 (lowest index among ties);
//   edges       4-neighbour pairs, key = (max(g2 p, g2 q), edge index) with
//               index 2p (p, p+1) and 2p+1 (p, p+W) — a strict total order;
//   forest      the minimum spanning forest relative to the markers.
//
// Marker components: union-find with hooking of the larger root onto the
// smaller (integer atomicMin), then pointer compression, until no edge joins
// two roots; each root ends as its component's smallest pixel.  Flooding:
// Boruvka rounds over the unmarked components — each picks its least
// outgoing edge (64-bit atomicMin on the key), hooks onto the component at
// the other end, mutual pairs keep the smaller id as root, and pointer
// jumping flattens the hooks.  With a strict edge order every picked edge
// belongs to the unique forest and the picks contain no cycle longer than
// two, so the labels do not depend on timing.  Marked components never
// pick, so every unmarked pixel ends in the tree of exactly one marker.
//
// Per-label sums for the scores are fixed-point integers: each value, scaled
// by a power of two S chosen from the largest |value| in the image so that no
// sum can exceed 2^92, is split as hi * 2^32 + lo (lo an integer in
// [0, 2^32]), and hi and lo are added into separate 64-bit integers with
// atomics.  Integer addition is associative, so the sums, and IRV and IRC,
// are the same bits on every run whatever the order of the adds; the
// quantum 1/S is about 2^-92 of the largest possible sum, far below FP64
// rounding of the same sums.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/abc.h"
#include "abc_internal.h"

namespace abc {
namespace {

constexpr int kT = 256;
constexpr int kRun = 16;  // pixels per thread in the per-label accumulations
constexpr unsigned long long kNoEdge = ~0ull;

enum Flag { kChanged = 0, kMarkers = 1, kActive = 2, kBadLabel = 3, kMaxLabel = 4, kNonEmpty = 5, kCount = 6,
            kAbsMax = 7, kFlags = 8 };

int nblocks(size_t n) { return (int)((n + kT - 1) / kT); }

__device__ __forceinline__ int ld(const int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Root of x under par (par[x] <= x always, so the walk ends).
__device__ __forceinline__ int find_root(const int* par, int x) {
    int y = ld(par + x);
    while (y != x) {
        x = y;
        y = ld(par + x);
    }
    return x;
}

__global__ void __launch_bounds__(kT)
relief_kernel(const float* __restrict__ c, int H, int W, int C, float th2, float* __restrict__ g2,
              unsigned char* __restrict__ mk, int* __restrict__ par, unsigned long long* __restrict__ minkey,
              int* __restrict__ flags) {
    const size_t N = (size_t)H * W;
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    unsigned long long key = kNoEdge;
    int m = 0;
    if (i < N) {
        const int r = (int)(i / W), q = (int)(i % W);
        float acc = 0.0f;
        for (int ch = 0; ch < C; ++ch) {
            float gx = 0.0f, gy = 0.0f;
            if (q >= 1 && q <= W - 2) gx = 0.5f * (c[(i + 1) * C + ch] - c[(i - 1) * C + ch]);
            if (r >= 1 && r <= H - 2) gy = 0.5f * (c[(i + W) * C + ch] - c[(i - W) * C + ch]);
            acc = fmaf(gx, gx, fmaf(gy, gy, acc));
        }
        g2[i] = acc;
        m = acc < th2;
        mk[i] = (unsigned char)m;
        par[i] = (int)i;
        key = ((unsigned long long)__float_as_uint(acc) << 32) | (unsigned long long)i;
    }
    // wave minimum of the (g2, index) keys and the marker count, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off, 64);
        key = o < key ? o : key;
        m += __shfl_xor(m, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(minkey, key);
        if (m) atomicAdd(&flags[kMarkers], m);
    }
}

// No pixel below the threshold: the lowest pixel becomes the only marker.
__global__ void fallback_marker_kernel(unsigned char* __restrict__ mk, const unsigned long long* __restrict__ minkey,
                                       const int* __restrict__ flags) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && flags[kMarkers] == 0) mk[(size_t)(*minkey & 0xffffffffull)] = 1;
}

__global__ void __launch_bounds__(kT)
cc_hook_kernel(const unsigned char* __restrict__ mk, int* par, int H, int W, int* __restrict__ flags) {
    const size_t N = (size_t)H * W;
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= N || !mk[i]) return;
    const int q = (int)(i % W);
    int changed = 0;
    for (int t = 0; t < 2; ++t) {
        size_t j;
        if (t == 0) {
            if (q + 1 >= W) continue;
            j = i + 1;
        } else {
            j = i + W;
            if (j >= N) continue;
        }
        if (!mk[j]) continue;
        const int a = find_root(par, (int)i), b = find_root(par, (int)j);
        if (a != b) {
            atomicMin(&par[a > b ? a : b], a < b ? a : b);
            changed = 1;
        }
    }
    if (changed) atomicOr(&flags[kChanged], 1);
}

__global__ void __launch_bounds__(kT)
cc_compress_kernel(const unsigned char* __restrict__ mk, int* par, size_t N) {
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= N || !mk[i]) return;
    const int r = find_root(par, (int)i);
    if (r != ld(par + i)) atomicMin(&par[i], r);
}

// comp: marker pixels -> their component root, others -> themselves.
__global__ void __launch_bounds__(kT)
forest_init_kernel(const unsigned char* __restrict__ mk, const int* __restrict__ par, int* __restrict__ comp,
                   size_t N) {
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i < N) comp[i] = mk[i] ? par[i] : (int)i;
}

__global__ void __launch_bounds__(kT)
round_init_kernel(unsigned long long* __restrict__ best, int* __restrict__ nxt, size_t N) {
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i < N) {
        best[i] = kNoEdge;
        nxt[i] = (int)i;
    }
}

// Least outgoing edge of every unmarked component.
__global__ void __launch_bounds__(kT)
select_kernel(const float* __restrict__ g2, const int* __restrict__ comp, const unsigned char* __restrict__ mk,
              unsigned long long* __restrict__ best, int H, int W) {
    const size_t N = (size_t)H * W;
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= N) return;
    const int cc = comp[i];
    if (mk[cc]) return;  // a component is marked iff its root pixel is a marker
    const int r = (int)(i / W), q = (int)(i % W);
    const float gi = g2[i];
    unsigned long long key = kNoEdge;
    const int nb[4] = {q > 0 ? (int)i - 1 : -1, q + 1 < W ? (int)i + 1 : -1, r > 0 ? (int)(i - W) : -1,
                       r + 1 < H ? (int)(i + W) : -1};
    for (int t = 0; t < 4; ++t) {
        const int j = nb[t];
        if (j < 0 || comp[j] == cc) continue;
        const float w = fmaxf(gi, g2[j]);
        const int lo = j < (int)i ? j : (int)i;
        const unsigned long long eid = 2ull * (unsigned long long)lo + (t >= 2 ? 1ull : 0ull);
        const unsigned long long k = ((unsigned long long)__float_as_uint(w) << 32) | eid;
        key = k < key ? k : key;
    }
    if (key != kNoEdge) atomicMin(&best[cc], key);
}

__global__ void __launch_bounds__(kT)
hook_kernel(const unsigned long long* __restrict__ best, const int* __restrict__ comp,
            const unsigned char* __restrict__ mk, int* __restrict__ nxt, int W, size_t N, int* __restrict__ flags) {
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= N || comp[i] != (int)i || mk[i] || best[i] == kNoEdge) return;
    const unsigned long long eid = best[i] & 0xffffffffull;
    const size_t p = (size_t)(eid >> 1);
    const size_t q = (eid & 1) ? p + W : p + 1;
    const int a = comp[p], b = comp[q];
    nxt[i] = a == (int)i ? b : a;
    atomicAdd(&flags[kActive], 1);
}

// Two unmarked components that picked each other (the same edge): the smaller id stays root.
__global__ void __launch_bounds__(kT)
pair_kernel(const int* __restrict__ comp, const unsigned char* __restrict__ mk, int* nxt, size_t N) {
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= N || comp[i] != (int)i || mk[i]) return;
    const int d = nxt[i];
    if (d != (int)i && nxt[d] == (int)i && (int)i < d) nxt[i] = (int)i;
}

__global__ void __launch_bounds__(kT)
jump_kernel(const int* __restrict__ comp, int* nxt, size_t N, int* __restrict__ flags) {
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= N || comp[i] != (int)i) return;
    const int n = ld(nxt + i);
    const int nn = ld(nxt + n);
    if (n != nn) {
        __hip_atomic_store(nxt + i, nn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicOr(&flags[kChanged], 1);
    }
}

__global__ void __launch_bounds__(kT)
relabel_kernel(int* __restrict__ comp, const int* __restrict__ nxt, size_t N) {
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i < N) comp[i] = nxt[comp[i]];
}

// Number the marker roots 0..k-1 in pixel order: per-block counts, a scan of
// the block counts, then per-block ranks.
__device__ __forceinline__ bool is_root(const unsigned char* mk, const int* par, size_t i) {
    return mk[i] && par[i] == (int)i;
}

__global__ void __launch_bounds__(kT)
count_roots_kernel(const unsigned char* __restrict__ mk, const int* __restrict__ par, size_t N,
                   int* __restrict__ bcount) {
    __shared__ int s[kT / 64];
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    const unsigned long long b = __ballot(i < N && is_root(mk, par, i));
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kT / 64; ++w) t += s[w];
        bcount[blockIdx.x] = t;
    }
}

// Exclusive scan of n block counts in place by one workgroup; total -> flags[kCount].
__global__ void __launch_bounds__(kT)
scan_blocks_kernel(int* __restrict__ bcount, int n, int* __restrict__ flags) {
    __shared__ int s[kT];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += kT) {
        const int idx = base + threadIdx.x;
        const int v = idx < n ? bcount[idx] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kT; off <<= 1) {
            const int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (idx < n) bcount[idx] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kT - 1) carry += s[kT - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) flags[kCount] = carry;
}

__global__ void __launch_bounds__(kT)
rank_roots_kernel(const unsigned char* __restrict__ mk, const int* __restrict__ par, size_t N,
                  const int* __restrict__ boff, int* __restrict__ id) {
    __shared__ int s[kT / 64];
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    const bool root = i < N && is_root(mk, par, i);
    const unsigned long long b = __ballot(root);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s[w] = __popcll(b);
    __syncthreads();
    int before = boff[blockIdx.x];
    for (int v = 0; v < w; ++v) before += s[v];
    const unsigned long long lower = lane ? (b & ((1ull << lane) - 1ull)) : 0ull;
    if (root) id[i] = before + __popcll(lower);
}

__global__ void __launch_bounds__(kT)
labels_kernel(const int* __restrict__ comp, const int* __restrict__ id, int* __restrict__ lab, size_t N) {
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i < N) lab[i] = id[comp[i]];
}

// Caller-supplied labels: range check and k = max + 1.
__global__ void __launch_bounds__(kT)
check_labels_kernel(const int* __restrict__ lab, size_t N, int* __restrict__ flags) {
    const size_t i = (size_t)blockIdx.x * kT + threadIdx.x;
    if (i >= N) return;
    const int l = lab[i];
    if (l < 0 || (size_t)l >= N)
        atomicOr(&flags[kBadLabel], 1);
    else
        atomicMax(&flags[kMaxLabel], l);
}

template <class T>
__global__ void __launch_bounds__(kT)
zero_kernel(T* __restrict__ x, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT) x[i] = T(0);
}

// Bit pattern of the largest |value| of c and c0 (as an int: the bits of a
// non-negative float order like integers, and those of NaN above infinity).
__global__ void __launch_bounds__(kT)
absmax_kernel(const float* __restrict__ c, const float* __restrict__ c0, size_t n, int* __restrict__ flags) {
    int m = 0;
    for (size_t i = (size_t)blockIdx.x * kT + threadIdx.x; i < n; i += (size_t)gridDim.x * kT) {
        m = max(m, __float_as_int(fabsf(c[i])));
        m = max(m, __float_as_int(fabsf(c0[i])));
    }
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(&flags[kAbsMax], m);
}

constexpr int kFxBits = 92;  // every sum stays below 2^kFxBits after scaling

// Scale 2^e with bound * 2^e < 2^kFxBits, bound = mult * (largest |value|);
// 0 when that value is not finite (the call then fails, see abc_segment).
__device__ __forceinline__ double fx_scale(const int* __restrict__ flags, double mult) {
    const float a = __int_as_float(flags[kAbsMax]);
    if (!(a <= 3.402823466e38f)) return 0.0;
    const double b = mult * (double)a;
    if (!(b > 0.0)) return 1.0;
    int e;
    (void)frexp(b, &e);  // b < 2^e
    return ldexp(1.0, kFxBits - e);
}

// Adds the scaled value v = x S as hi * 2^32 + lo: hi = floor(v / 2^32) and
// lo = v - hi 2^32 rounded to an integer in [0, 2^32].
__device__ __forceinline__ void fx_add(double v, long long& hi, unsigned long long& lo) {
    const double h = floor(v * 0x1p-32);
    hi += (long long)h;
    lo += (unsigned long long)rint(fma(h, -0x1p32, v));
}

__device__ __forceinline__ void fx_flush(unsigned long long* __restrict__ dst, long long hi, unsigned long long lo) {
    atomicAdd(dst, (unsigned long long)hi);  // two's complement: the wrapped sum is the signed one
    atomicAdd(dst + 1, lo);
}

// Value of a fixed-point sum, still scaled by S.
__device__ __forceinline__ double fx_value(const unsigned long long* __restrict__ x) {
    return fma((double)(long long)x[0], 0x1p32, (double)x[1]);
}

// Per-label pixel count (FP64 integer sums, exact) and fixed-point channel
// sums of c0 and c (pairs hi, lo at s0[2 (label C + ch)]), one run of kRun
// pixels per thread, flushed with atomics whenever the label changes.
__global__ void __launch_bounds__(kT)
label_sums_kernel(const float* __restrict__ c, const float* __restrict__ c0, const int* __restrict__ lab, size_t N,
                  int C, const int* __restrict__ flags, double* __restrict__ cnt, unsigned long long* __restrict__ s0,
                  unsigned long long* __restrict__ s1) {
    const size_t p0 = ((size_t)blockIdx.x * kT + threadIdx.x) * kRun;
    const double S = fx_scale(flags, (double)N);
    if (p0 >= N || S == 0.0) return;
    const size_t p1 = p0 + kRun < N ? p0 + kRun : N;
    int cur = lab[p0];
    double n = 0.0;
    for (size_t i = p0; i < p1; ++i) {
        const int l = lab[i];
        if (l != cur) {
            atomicAdd(&cnt[cur], n);
            cur = l;
            n = 0.0;
        }
        n += 1.0;
    }
    atomicAdd(&cnt[cur], n);
    for (int ch = 0; ch < C; ++ch) {
        cur = lab[p0];
        long long h0 = 0, h1 = 0;
        unsigned long long l0 = 0, l1 = 0;
        for (size_t i = p0; i < p1; ++i) {
            const int l = lab[i];
            if (l != cur) {
                fx_flush(s0 + 2 * ((size_t)cur * C + ch), h0, l0);
                fx_flush(s1 + 2 * ((size_t)cur * C + ch), h1, l1);
                cur = l;
                h0 = h1 = 0;
                l0 = l1 = 0;
            }
            fx_add((double)c0[i * C + ch] * S, h0, l0);
            fx_add((double)c[i * C + ch] * S, h1, l1);
        }
        fx_flush(s0 + 2 * ((size_t)cur * C + ch), h0, l0);
        fx_flush(s1 + 2 * ((size_t)cur * C + ch), h1, l1);
    }
}

// Label means m0, m1 of c0 and c from the fixed-point sums.
__global__ void __launch_bounds__(kT)
label_means_kernel(const double* __restrict__ cnt, const unsigned long long* __restrict__ s0,
                   const unsigned long long* __restrict__ s1, size_t N, int k, int C, int* __restrict__ flags,
                   double* __restrict__ m0, double* __restrict__ m1) {
    const int j = blockIdx.x * kT + threadIdx.x;
    if (j >= k) return;
    const double S = fx_scale(flags, (double)N);
    const double n = cnt[j];
    if (n > 0.0 && S != 0.0) {
        atomicAdd(&flags[kNonEmpty], 1);
        for (int ch = 0; ch < C; ++ch) {
            const size_t e = (size_t)j * C + ch;
            m0[e] = fx_value(s0 + 2 * e) / S / n;
            m1[e] = fx_value(s1 + 2 * e) / S / n;
        }
    }
}

// Squared deviations of c0 from its label means, per label in fixed point
// (pairs hi, lo), with the bound 4 C (largest |value|)^2 per pixel.
__global__ void __launch_bounds__(kT)
label_dev_kernel(const float* __restrict__ c0, const int* __restrict__ lab, size_t N, int C,
                 const int* __restrict__ flags, const double* __restrict__ m0, unsigned long long* __restrict__ dev) {
    const size_t p0 = ((size_t)blockIdx.x * kT + threadIdx.x) * kRun;
    const float a = __int_as_float(flags[kAbsMax]);
    const double S = fx_scale(flags, 4.0 * (double)N * (double)C * (double)a);
    if (p0 >= N || S == 0.0) return;
    const size_t p1 = p0 + kRun < N ? p0 + kRun : N;
    int cur = lab[p0];
    long long h = 0;
    unsigned long long lo = 0;
    for (size_t i = p0; i < p1; ++i) {
        const int l = lab[i];
        if (l != cur) {
            fx_flush(dev + 2 * (size_t)cur, h, lo);
            cur = l;
            h = 0;
            lo = 0;
        }
        double t = 0.0;
        for (int ch = 0; ch < C; ++ch) {
            const double d = (double)c0[i * C + ch] - m0[(size_t)l * C + ch];
            t = fma(d, d, t);
        }
        fx_add(t * S, h, lo);
    }
    fx_flush(dev + 2 * (size_t)cur, h, lo);
}

// IRV = sum_j dev_j / N: integer sums of the hi and lo words over the labels
// by one workgroup (exact, so their order is immaterial), then one conversion.
__global__ void __launch_bounds__(kT)
irv_kernel(const unsigned long long* __restrict__ dev, int k, size_t N, int C, const int* __restrict__ flags,
           double* __restrict__ out) {
    __shared__ unsigned long long s[2][kT];
    unsigned long long h = 0, lo = 0;
    for (int j = threadIdx.x; j < k; j += kT) {
        h += dev[2 * (size_t)j];
        lo += dev[2 * (size_t)j + 1];
    }
    s[0][threadIdx.x] = h;
    s[1][threadIdx.x] = lo;
    __syncthreads();
    for (int off = kT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s[0][threadIdx.x] += s[0][threadIdx.x + off];
            s[1][threadIdx.x] += s[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float a = __int_as_float(flags[kAbsMax]);
        const double S = fx_scale(flags, 4.0 * (double)N * (double)C * (double)a);
        const unsigned long long t[2] = {s[0][0], s[1][0]};
        *out = S == 0.0 ? NAN : fx_value(t) / S / (double)N;
    }
}

// IRC: least distance between the mean colours of two non-empty labels.
// Thread pairs (a, b > a) over a grid-stride loop on a; the minimum is taken
// on the bit patterns of the (non-negative) FP64 distances.
__global__ void __launch_bounds__(kT)
irc_kernel(const double* __restrict__ cnt, const double* __restrict__ m1, int k, int C,
           unsigned long long* __restrict__ best) {
    unsigned long long mine = kNoEdge;
    for (size_t t = (size_t)blockIdx.x * kT + threadIdx.x; t < (size_t)k * k; t += (size_t)gridDim.x * kT) {
        const int a = (int)(t / k), b = (int)(t % k);
        if (b <= a || cnt[a] == 0.0 || cnt[b] == 0.0) continue;
        double s = 0.0;
        for (int ch = 0; ch < C; ++ch) {
            const double d = m1[(size_t)a * C + ch] - m1[(size_t)b * C + ch];
            s = fma(d, d, s);
        }
        const unsigned long long bits = (unsigned long long)__double_as_longlong(sqrt(s));
        mine = bits < mine ? bits : mine;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(mine, off, 64);
        mine = o < mine ? o : mine;
    }
    if ((threadIdx.x & 63) == 0 && mine != kNoEdge) atomicMin(best, mine);
}

__global__ void set_u64_kernel(unsigned long long* x, unsigned long long v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *x = v;
}

__global__ void clear_flags_kernel(int* flags, int n) {
    if ((int)threadIdx.x < n) flags[threadIdx.x] = 0;
}

// Workspace layout (every piece 256-byte aligned).
struct SegWs {
    float* g2;
    unsigned char* mk;
    int* par;
    int* comp;
    int* nxt;
    int* lab;
    int* bcount;
    int* flags;
    unsigned long long* best;
    unsigned long long* keys;  // [0] min (g2, index) key, [1] IRC bits
    double* cnt;
    unsigned long long* s0;  // fixed-point pairs (hi, lo) per label and channel
    unsigned long long* s1;
    double* m0;              // label means
    double* m1;
    unsigned long long* dev;  // fixed-point pairs per label
    double* irv;
    size_t bytes;
};

size_t al(size_t x) { return (x + 255) / 256 * 256; }

SegWs carve(void* base, int H, int W, int C) {
    const size_t N = (size_t)H * W;
    SegWs w{};
    char* b = (char*)base;
    size_t o = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = b ? b + o : nullptr;
        o += al(bytes);
        return p;
    };
    w.g2 = (float*)take(N * sizeof(float));
    w.mk = (unsigned char*)take(N);
    w.par = (int*)take(N * sizeof(int));
    w.comp = (int*)take(N * sizeof(int));
    w.nxt = (int*)take(N * sizeof(int));
    w.lab = (int*)take(N * sizeof(int));
    w.bcount = (int*)take((size_t)nblocks(N) * sizeof(int));
    w.flags = (int*)take(kFlags * sizeof(int));
    w.best = (unsigned long long*)take(N * sizeof(unsigned long long));
    w.keys = (unsigned long long*)take(2 * sizeof(unsigned long long));
    w.cnt = (double*)take(N * sizeof(double));
    w.s0 = (unsigned long long*)take(2 * N * (size_t)C * sizeof(unsigned long long));
    w.s1 = (unsigned long long*)take(2 * N * (size_t)C * sizeof(unsigned long long));
    w.m0 = (double*)take(N * (size_t)C * sizeof(double));
    w.m1 = (double*)take(N * (size_t)C * sizeof(double));
    w.dev = (unsigned long long*)take(2 * N * sizeof(unsigned long long));
    w.irv = (double*)take(sizeof(double));
    w.bytes = o;
    return w;
}

#define SEG_HIP(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            set_last_error(std::string(#expr) + ": " + hipGetErrorString(e_));                      \
            return ABC_EHIP;                                                                        \
        }                                                                                           \
    } while (0)

#define SEG_LAUNCH(kernel, grid, ...)                                                               \
    do {                                                                                            \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kT), 0, st, __VA_ARGS__);                       \
        SEG_HIP(hipGetLastError());                                                                 \
    } while (0)

// Pinned host staging for the reads the round loop waits on: one per host
// thread, allocated on its first use and kept until the process ends (a read
// into pinned memory returns several microseconds sooner than one into
// pageable memory, and the loop waits on one per round).  Layout: the flags,
// then the IRV double and the IRC bit pattern.  NULL if the allocation failed.
struct SegReadback {
    int flags[kFlags];
    double irv;
    unsigned long long ircbits;
};
SegReadback* seg_readback() {
    thread_local SegReadback* buf = nullptr;
    thread_local bool tried = false;
    if (!tried) {
        tried = true;
        if (hipHostMalloc((void**)&buf, sizeof(SegReadback), hipHostMallocDefault) != hipSuccess) {
            buf = nullptr;
            (void)hipGetLastError();
        }
    }
    return buf;
}

int read_flags(int* dst, const int* flags, hipStream_t st) {
    SegReadback* pin = seg_readback();
    int* to = pin ? pin->flags : dst;
    SEG_HIP(hipMemcpyAsync(to, flags, kFlags * sizeof(int), hipMemcpyDeviceToHost, st));
    SEG_HIP(hipStreamSynchronize(st));
    if (pin) std::memcpy(dst, pin->flags, kFlags * sizeof(int));
    return ABC_OK;
}

constexpr int kMaxIterations = 4096;

}  // namespace
}  // namespace abc

extern "C" {

int abc_segment_workspace_bytes(int H, int W, int C, size_t* bytes) {
    if (!bytes || H < 1 || W < 1 || C < 1 || C > ABC_MAX_CHANNELS || (size_t)H * W >= (1ull << 31)) {
        abc::set_last_error("abc_segment_workspace_bytes: bad shape or null output");
        return ABC_EINVAL;
    }
    *bytes = abc::carve(nullptr, H, W, C).bytes;
    return ABC_OK;
}

int abc_segment(const float* c, const float* c0, int H, int W, int C, float theta, const int32_t* labels_in,
                int32_t* labels_out, abc_seg_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    using namespace abc;
    if (!c || !c0 || !stats || !ws || H < 1 || W < 1 || C < 1 || C > ABC_MAX_CHANNELS ||
        (size_t)H * W >= (1ull << 31) || !std::isfinite(theta)) {
        set_last_error("abc_segment: null pointer, bad shape or non-finite theta");
        return ABC_EINVAL;
    }
    const SegWs w = carve(ws, H, W, C);
    if (ws_bytes < w.bytes) {
        set_last_error("abc_segment: workspace too small (need " + std::to_string(w.bytes) + " bytes)");
        return ABC_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    const size_t N = (size_t)H * W;
    const int nb = nblocks(N);
    int f[kFlags];
    int rc;
    abc_seg_stats out{};
    const int* lab = labels_in;
    int k = 0;
    SEG_LAUNCH(clear_flags_kernel, 1, w.flags, (int)kFlags);
    const int ab = (int)std::min<size_t>((size_t)nblocks(N * C), 2048);
    SEG_LAUNCH(absmax_kernel, ab, c, c0, N * C, w.flags);
    if ((rc = read_flags(f, w.flags, st)) != ABC_OK) return rc;
    if (f[kAbsMax] >= 0x7f800000) {
        set_last_error("abc_segment: c or c0 holds a NaN or an infinity");
        return ABC_ENONFINITE;
    }
    if (!labels_in) {
        SEG_LAUNCH(set_u64_kernel, 1, w.keys, kNoEdge);
        SEG_LAUNCH(relief_kernel, nb, c, H, W, C, theta * theta, w.g2, w.mk, w.par, w.keys, w.flags);
        SEG_LAUNCH(fallback_marker_kernel, 1, w.mk, (const unsigned long long*)w.keys, (const int*)w.flags);
        // marker components
        int it = 0;
        for (;; ++it) {
            if (it >= kMaxIterations) {
                set_last_error("abc_segment: marker components did not settle");
                return ABC_EHIP;
            }
            SEG_LAUNCH(clear_flags_kernel, 1, w.flags, 1);
            SEG_LAUNCH(cc_hook_kernel, nb, (const unsigned char*)w.mk, w.par, H, W, w.flags);
            SEG_LAUNCH(cc_compress_kernel, nb, (const unsigned char*)w.mk, w.par, N);
            if ((rc = read_flags(f, w.flags, st)) != ABC_OK) return rc;
            if (!f[kChanged]) break;
        }
        // flooding
        SEG_LAUNCH(forest_init_kernel, nb, (const unsigned char*)w.mk, (const int*)w.par, w.comp, N);
        int rounds = 0;
        for (;; ++rounds) {
            if (rounds >= 64) {
                set_last_error("abc_segment: flooding did not finish in 64 rounds");
                return ABC_EHIP;
            }
            SEG_LAUNCH(round_init_kernel, nb, w.best, w.nxt, N);
            SEG_LAUNCH(clear_flags_kernel, 1, w.flags, (int)kFlags);
            SEG_LAUNCH(select_kernel, nb, (const float*)w.g2, (const int*)w.comp, (const unsigned char*)w.mk, w.best,
                       H, W);
            SEG_LAUNCH(hook_kernel, nb, (const unsigned long long*)w.best, (const int*)w.comp,
                       (const unsigned char*)w.mk, w.nxt, W, N, w.flags);
            if ((rc = read_flags(f, w.flags, st)) != ABC_OK) return rc;
            if (f[kActive] == 0) break;
            SEG_LAUNCH(pair_kernel, nb, (const int*)w.comp, (const unsigned char*)w.mk, w.nxt, N);
            for (int j = 0;; ++j) {
                if (j >= 64) {
                    set_last_error("abc_segment: pointer jumping did not settle");
                    return ABC_EHIP;
                }
                SEG_LAUNCH(clear_flags_kernel, 1, w.flags, 1);
                SEG_LAUNCH(jump_kernel, nb, (const int*)w.comp, w.nxt, N, w.flags);
                if ((rc = read_flags(f, w.flags, st)) != ABC_OK) return rc;
                if (!f[kChanged]) break;
            }
            SEG_LAUNCH(relabel_kernel, nb, w.comp, (const int*)w.nxt, N);
        }
        out.rounds = rounds;
        // number the marker roots in pixel order, then label every pixel
        SEG_LAUNCH(count_roots_kernel, nb, (const unsigned char*)w.mk, (const int*)w.par, N, w.bcount);
        hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kT), 0, st, w.bcount, nb, w.flags);
        SEG_HIP(hipGetLastError());
        SEG_LAUNCH(rank_roots_kernel, nb, (const unsigned char*)w.mk, (const int*)w.par, N, (const int*)w.bcount,
                   w.nxt);
        int* dst = labels_out ? labels_out : w.lab;
        SEG_LAUNCH(labels_kernel, nb, (const int*)w.comp, (const int*)w.nxt, dst, N);
        if ((rc = read_flags(f, w.flags, st)) != ABC_OK) return rc;
        k = f[kCount];
        lab = dst;
    } else {
        SEG_LAUNCH(check_labels_kernel, nb, labels_in, N, w.flags);
        if ((rc = read_flags(f, w.flags, st)) != ABC_OK) return rc;
        if (f[kBadLabel]) {
            set_last_error("abc_segment: a label lies outside [0, H*W)");
            return ABC_EINVAL;
        }
        k = f[kMaxLabel] + 1;
    }
    out.k = k;
    // scores
    const int zb = 1024;
    SEG_LAUNCH(zero_kernel<double>, zb, w.cnt, (size_t)k);
    SEG_LAUNCH(zero_kernel<unsigned long long>, zb, w.s0, 2 * (size_t)k * C);
    SEG_LAUNCH(zero_kernel<unsigned long long>, zb, w.s1, 2 * (size_t)k * C);
    SEG_LAUNCH(zero_kernel<unsigned long long>, zb, w.dev, 2 * (size_t)k);
    SEG_LAUNCH(clear_flags_kernel, 1, w.flags, (int)kFlags);
    SEG_LAUNCH(set_u64_kernel, 1, w.keys + 1, kNoEdge);
    SEG_LAUNCH(absmax_kernel, ab, c, c0, N * C, w.flags);  // the fixed-point scales
    const int nr = nblocks((N + kRun - 1) / kRun);
    SEG_LAUNCH(label_sums_kernel, nr, c, c0, lab, N, C, (const int*)w.flags, w.cnt, w.s0, w.s1);
    SEG_LAUNCH(label_means_kernel, nblocks((size_t)k), (const double*)w.cnt, (const unsigned long long*)w.s0,
               (const unsigned long long*)w.s1, N, k, C, w.flags, w.m0, w.m1);
    SEG_LAUNCH(label_dev_kernel, nr, c0, lab, N, C, (const int*)w.flags, (const double*)w.m0, w.dev);
    hipLaunchKernelGGL(irv_kernel, dim3(1), dim3(kT), 0, st, (const unsigned long long*)w.dev, k, N, C,
                       (const int*)w.flags, w.irv);
    SEG_HIP(hipGetLastError());
    const size_t pairs = (size_t)k * k;
    const int gb = (int)std::min<size_t>(std::max<size_t>((pairs + kT - 1) / kT, 1), 8192);
    SEG_LAUNCH(irc_kernel, gb, (const double*)w.cnt, (const double*)w.m1, k, C, w.keys + 1);
    unsigned long long ircbits = 0;
    double irv = 0.0;
    SegReadback* pin = seg_readback();
    SEG_HIP(hipMemcpyAsync(pin ? &pin->irv : &irv, w.irv, sizeof(double), hipMemcpyDeviceToHost, st));
    SEG_HIP(hipMemcpyAsync(pin ? &pin->ircbits : &ircbits, w.keys + 1, sizeof(ircbits), hipMemcpyDeviceToHost, st));
    if ((rc = read_flags(f, w.flags, st)) != ABC_OK) return rc;
    if (pin) {
        irv = pin->irv;
        ircbits = pin->ircbits;
    }
    out.nonempty = f[kNonEmpty];
    out.irv = irv;
    if (out.nonempty < 2) {
        out.irc = NAN;
    } else {
        double d;
        std::memcpy(&d, &ircbits, sizeof d);
        out.irc = d;
    }
    out.vs = out.irv / out.irc;
    *stats = out;
    return ABC_OK;
}

}  // extern "C"
