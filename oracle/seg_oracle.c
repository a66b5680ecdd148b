/*
 * CPU oracle of the segmentation metrics of Sec. 4.4 (intra-region variance,
 * inter-region contrast, validity score) and of the watershed labelling they
 * are computed on.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library and must never be used as a
 * fallback for it.
 *
 * The paper labels the segments of a processed image with the watershed
 * algorithm at threshold 0.02 and gives no further detail.  The labelling
 * here is the marker-based watershed defined as a minimum spanning forest:
 *
 *  relief   g2(p) = sum over channels of gx^2 + gy^2 with the central
 *           differences of Def. 3.1 in pixel units, gx = (c(q+1) - c(q-1))/2,
 *           zero on the first and last column (same for gy along rows).
 *           It is evaluated in FP32 in a fixed order: per channel, ascending,
 *           g2 = fma(gx, gx, fma(gy, gy, g2)), so that every comparison below
 *           is taken on the same FP32 values as on the GPU;
 *  markers  the 4-connected components of {p : g2(p) < theta*theta}
 *           (theta*theta rounded to FP32); if no pixel qualifies, the pixel
 *           of smallest g2 (lowest index among ties) is the only marker;
 *  edges    4-neighbour pairs; the horizontal edge from p to p+1 has index
 *           2p, the vertical edge from p to p+W has index 2p+1; its weight is
 *           max(g2(p), g2(q)) and edges are ordered by (weight, index);
 *  flooding Kruskal's algorithm over the ordered edges where each marker
 *           component starts as one labelled set and two labelled sets are
 *           never joined: the unique minimum spanning forest relative to the
 *           markers.  A pixel's label is its tree's marker component.
 *  labels   markers are numbered 0..k-1 in increasing order of their
 *           smallest pixel index.
 *
 * The metrics follow their definitions in Sec. 4.4 for colour fields:
 *   IRV = (1/N) sum_j sum_{p in R_j} |c0_p - mean0_j|^2  (original image),
 *   IRC = min_{i<j} |mean_i - mean_j|                    (processed image),
 *   VS  = IRV / IRC,
 * with |.| the Euclidean norm over channels (the variance of a colour region
 * is the sum of its per-channel variances).  Empty labels are ignored; with
 * fewer than two non-empty labels IRC and VS are NaN.  FP64 throughout.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SEG_OK 0
#define SEG_EINVAL (-1)
#define SEG_ENOMEM (-4)

/* FP32 relief of the processed field c (H x W x C, float, channel fastest). */
void seg_relief(const float* c, int H, int W, int C, float* g2)
{
    for (int r = 0; r < H; ++r) {
        for (int q = 0; q < W; ++q) {
            const size_t i = (size_t)r * W + q;
            float acc = 0.0f;
            for (int ch = 0; ch < C; ++ch) {
                float gx = 0.0f, gy = 0.0f;
                if (q >= 1 && q <= W - 2) {
                    const float d = c[(i + 1) * C + ch] - c[(i - 1) * C + ch];
                    gx = 0.5f * d;
                }
                if (r >= 1 && r <= H - 2) {
                    const float d = c[(i + W) * C + ch] - c[(i - W) * C + ch];
                    gy = 0.5f * d;
                }
                acc = fmaf(gx, gx, fmaf(gy, gy, acc));
            }
            g2[i] = acc;
        }
    }
}

/* union-find with path halving; the root carries the set's label (-1: none) */
static int uf_find(int* parent, int x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

typedef struct {
    float w;
    uint32_t id;
} seg_edge;

static int edge_cmp(const void* a, const void* b)
{
    const seg_edge* x = (const seg_edge*)a;
    const seg_edge* y = (const seg_edge*)b;
    if (x->w < y->w) return -1;
    if (x->w > y->w) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* Watershed labels of c (see the file comment).  labels: H*W int32 output.
 * Returns the number of labels k (>= 1), or a negative error. */
int seg_watershed(const float* c, int H, int W, int C, float theta, int32_t* labels)
{
    if (!c || !labels || H < 1 || W < 1 || C < 1) return SEG_EINVAL;
    const size_t N = (size_t)H * W;
    float* g2 = (float*)malloc(N * sizeof(float));
    int* parent = (int*)malloc(N * sizeof(int));
    int* lab = (int*)malloc(N * sizeof(int));
    int* stack = (int*)malloc(N * sizeof(int));
    size_t ne = (size_t)H * (W - 1) + (size_t)(H - 1) * W;
    seg_edge* edges = (seg_edge*)malloc((ne ? ne : 1) * sizeof(seg_edge));
    if (!g2 || !parent || !lab || !stack || !edges) {
        free(g2); free(parent); free(lab); free(stack); free(edges);
        return SEG_ENOMEM;
    }
    seg_relief(c, H, W, C, g2);
    const float th2 = theta * theta;

    /* markers */
    size_t nmark = 0;
    for (size_t i = 0; i < N; ++i) nmark += g2[i] < th2;
    char* mark = (char*)calloc(N, 1);
    if (!mark) {
        free(g2); free(parent); free(lab); free(stack); free(edges);
        return SEG_ENOMEM;
    }
    if (nmark == 0) {
        size_t best = 0;
        for (size_t i = 1; i < N; ++i)
            if (g2[i] < g2[best]) best = i;
        mark[best] = 1;
    } else {
        for (size_t i = 0; i < N; ++i) mark[i] = g2[i] < th2;
    }

    /* marker components by depth-first search, numbered in the order of their
     * smallest pixel (the scan meets that pixel first) */
    for (size_t i = 0; i < N; ++i) lab[i] = -1;
    int k = 0;
    for (size_t s = 0; s < N; ++s) {
        if (!mark[s] || lab[s] >= 0) continue;
        size_t top = 0;
        stack[top++] = (int)s;
        lab[s] = k;
        while (top > 0) {
            const int p = stack[--top];
            const int r = p / W, q = p % W;
            const int nb[4][2] = {{r, q - 1}, {r, q + 1}, {r - 1, q}, {r + 1, q}};
            for (int t = 0; t < 4; ++t) {
                const int rr = nb[t][0], qq = nb[t][1];
                if (rr < 0 || rr >= H || qq < 0 || qq >= W) continue;
                const int j = rr * W + qq;
                if (mark[j] && lab[j] < 0) {
                    lab[j] = k;
                    stack[top++] = j;
                }
            }
        }
        ++k;
    }

    /* union-find: one set per marker component (rooted at its first pixel),
     * singletons elsewhere */
    int* first = (int*)malloc((size_t)k * sizeof(int));
    if (!first) {
        free(g2); free(parent); free(lab); free(stack); free(edges); free(mark);
        return SEG_ENOMEM;
    }
    for (int j = 0; j < k; ++j) first[j] = -1;
    for (size_t i = 0; i < N; ++i) {
        parent[i] = (int)i;
        if (lab[i] >= 0) {
            if (first[lab[i]] < 0)
                first[lab[i]] = (int)i;
            else
                parent[i] = first[lab[i]];
        }
    }

    /* edges ordered by (weight, index) */
    size_t m = 0;
    for (int r = 0; r < H; ++r)
        for (int q = 0; q < W; ++q) {
            const size_t p = (size_t)r * W + q;
            if (q + 1 < W) {
                edges[m].w = fmaxf(g2[p], g2[p + 1]);
                edges[m].id = (uint32_t)(2 * p);
                ++m;
            }
            if (r + 1 < H) {
                edges[m].w = fmaxf(g2[p], g2[p + W]);
                edges[m].id = (uint32_t)(2 * p + 1);
                ++m;
            }
        }
    qsort(edges, m, sizeof(seg_edge), edge_cmp);

    /* Kruskal relative to the markers; lab[root] is the set's label */
    for (size_t e = 0; e < m; ++e) {
        const size_t p = edges[e].id / 2;
        const size_t q = (edges[e].id & 1) ? p + W : p + 1;
        const int a = uf_find(parent, (int)p), b = uf_find(parent, (int)q);
        if (a == b) continue;
        if (lab[a] >= 0 && lab[b] >= 0) continue;
        if (lab[a] >= 0) {
            parent[b] = a;
        } else {
            parent[a] = b;
        }
    }
    for (size_t i = 0; i < N; ++i) labels[i] = lab[uf_find(parent, (int)i)];

    free(g2); free(parent); free(lab); free(stack); free(edges); free(mark); free(first);
    return k;
}

/* IRV, IRC, VS (out[0..2]) of a labelling with labels in [0, k).  c is the
 * processed field, c0 the original image (both H x W x C float).  Returns 0,
 * or SEG_EINVAL when a label lies outside [0, k). */
int seg_metrics(const float* c, const float* c0, const int32_t* labels, int H, int W, int C, int k,
                double* out)
{
    if (!c || !c0 || !labels || !out || H < 1 || W < 1 || C < 1 || k < 1) return SEG_EINVAL;
    const size_t N = (size_t)H * W;
    for (size_t i = 0; i < N; ++i)
        if (labels[i] < 0 || labels[i] >= k) return SEG_EINVAL;
    double* cnt = (double*)calloc((size_t)k, sizeof(double));
    double* m0 = (double*)calloc((size_t)k * C, sizeof(double));
    double* m1 = (double*)calloc((size_t)k * C, sizeof(double));
    if (!cnt || !m0 || !m1) {
        free(cnt); free(m0); free(m1);
        return SEG_ENOMEM;
    }
    for (size_t i = 0; i < N; ++i) {
        const int j = labels[i];
        cnt[j] += 1.0;
        for (int ch = 0; ch < C; ++ch) {
            m0[(size_t)j * C + ch] += (double)c0[i * C + ch];
            m1[(size_t)j * C + ch] += (double)c[i * C + ch];
        }
    }
    for (int j = 0; j < k; ++j)
        for (int ch = 0; ch < C; ++ch)
            if (cnt[j] > 0) {
                m0[(size_t)j * C + ch] /= cnt[j];
                m1[(size_t)j * C + ch] /= cnt[j];
            }
    /* IRV: sum over regions of |R_j| sigma_j^2 = sum of squared deviations */
    double irv = 0.0;
    for (size_t i = 0; i < N; ++i) {
        const int j = labels[i];
        for (int ch = 0; ch < C; ++ch) {
            const double d = (double)c0[i * C + ch] - m0[(size_t)j * C + ch];
            irv += d * d;
        }
    }
    irv /= (double)N;
    /* IRC: smallest distance between the mean colours of two regions */
    double irc = INFINITY;
    int nonempty = 0;
    for (int a = 0; a < k; ++a) {
        if (cnt[a] == 0) continue;
        ++nonempty;
        for (int b = a + 1; b < k; ++b) {
            if (cnt[b] == 0) continue;
            double s = 0.0;
            for (int ch = 0; ch < C; ++ch) {
                const double d = m1[(size_t)a * C + ch] - m1[(size_t)b * C + ch];
                s += d * d;
            }
            const double dist = sqrt(s);
            if (dist < irc) irc = dist;
        }
    }
    if (nonempty < 2) irc = NAN;
    out[0] = irv;
    out[1] = irc;
    out[2] = irv / irc;
    free(cnt); free(m0); free(m1);
    return SEG_OK;
}
