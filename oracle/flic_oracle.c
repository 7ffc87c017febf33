/*
 * flic_oracle.c -- CPU oracle for FLIC range-image clustering.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.  Shares no code with
 * the GPU library.
 *
 * It computes the plain definition: build every edge of the neighbour graph
 * in one raster pass (Section III.B, Eq. 4, with the dense skip connections
 * of Section III.B.2), then label each connected component by breadth-first
 * search seeded in raster order, so the seed -- the first pixel of its
 * component in raster order -- is the component's minimum linear index.
 * The cluster-size threshold of Section III.B.1 is a separate step on those
 * labels: count the pixels of every label, then drop the small labels.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (x86-64 SSE float math:
 * every float operation is one IEEE binary32 rounding).
 */
#include "flic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Section III.A: a range of zero is a missing measurement; negative, NaN and
 * infinite values are treated the same way. */
static int is_measurement(float r) { return r > 0.0f && r < INFINITY; }

/* Section III.B, Eq. (4): four multiplications, one addition, one
 * subtraction, with 2*cos(alpha) as the precomputed constant. */
float flic_oracle_dist2(float d1, float d2, float cos_alpha) {
    float two_cos = 2.0f * cos_alpha;
    float sq1 = d1 * d1;
    float sq2 = d2 * d2;
    float sum = sq1 + sq2;
    float prod = d1 * d2;
    float cross = two_cos * prod;
    return sum - cross;
}

/* Edge test: both pixels are measurements and D^2 <= T^2 (ordered compare,
 * so a NaN distance never connects). */
static int connected(float d1, float d2, float cos_alpha, float t2) {
    if (!is_measurement(d1) || !is_measurement(d2)) return 0;
    float d2sq = flic_oracle_dist2(d1, d2, cos_alpha);
    return d2sq <= t2;
}

/* Section III.B.2, the paper's own Map Connections: a map of stride k holds
 * the points whose row and column are both multiples of k, and connects each
 * with its k-th neighbour to the right and below.  A skip edge of offset k is
 * present only when its first end (the upper or left one) lies on that map. */
static int on_map(int32_t r, int32_t c, int32_t k) { return r % k == 0 && c % k == 0; }

int32_t flic_oracle_cluster_maps(const float* range, int32_t H, int32_t W,
                                 const float* cos_v, const float* cos_h,
                                 float threshold, int32_t skip_depth, int32_t maps,
                                 int32_t* labels_out);

int32_t flic_oracle_cluster(const float* range, int32_t H, int32_t W,
                            const float* cos_v, const float* cos_h,
                            float threshold, int32_t skip_depth,
                            int32_t* labels_out) {
    return flic_oracle_cluster_maps(range, H, W, cos_v, cos_h, threshold, skip_depth, 0, labels_out);
}

int32_t flic_oracle_cluster_maps(const float* range, int32_t H, int32_t W,
                                 const float* cos_v, const float* cos_h,
                                 float threshold, int32_t skip_depth, int32_t maps,
                                 int32_t* labels_out) {
    if (maps != 0 && maps != 1) return -1;
    if (!range || !cos_v || !cos_h || !labels_out) return -1;
    if (H < 1 || W < 1) return -1;
    if (skip_depth < 1 || skip_depth > 8) return -1;
    if (2 * skip_depth >= W) return -1;
    if ((int64_t)H * (int64_t)W > (int64_t)INT32_MAX) return -1;
    if (!(threshold >= 0.0f) || !(threshold < INFINITY)) return -1;
    {
        const char* a0 = (const char*)range;
        const char* a1 = a0 + (size_t)H * W * sizeof(float);
        const char* b0 = (const char*)labels_out;
        const char* b1 = b0 + (size_t)H * W * sizeof(int32_t);
        if (a0 < b1 && b0 < a1) return -1;
    }

    const int32_t N = skip_depth;
    const size_t P = (size_t)H * (size_t)W;
    const float t2 = threshold * threshold;

    /* Pass 1: every undirected edge exactly once, in raster order. */
    size_t cap = 2u * (size_t)N * P, ne = 0;
    int32_t* eu = (int32_t*)malloc(cap * sizeof(int32_t));
    int32_t* ev = (int32_t*)malloc(cap * sizeof(int32_t));
    if (!eu || !ev) { free(eu); free(ev); return -2; }
    for (int32_t r = 0; r < H; ++r) {
        for (int32_t c = 0; c < W; ++c) {
            const int32_t p = r * W + c;
            for (int32_t k = 1; k <= N; ++k) {
                if (maps && k >= 2 && !on_map(r, c, k)) continue;
                /* vertical: (r, c) -- (r+k, c), angle between rows r, r+k */
                if (r + k < H) {
                    const int32_t q = p + k * W;
                    if (connected(range[p], range[q], cos_v[(size_t)(k - 1) * H + r], t2)) {
                        eu[ne] = p; ev[ne] = q; ++ne;
                    }
                }
                /* horizontal with 360-degree wrap: (r, c) -- (r, (c+k) mod W) */
                {
                    const int32_t q = r * W + (c + k) % W;
                    if (connected(range[p], range[q], cos_h[(size_t)(k - 1) * W + c], t2)) {
                        eu[ne] = p; ev[ne] = q; ++ne;
                    }
                }
            }
        }
    }

    /* Adjacency lists (CSR) of the undirected graph. */
    size_t* off = (size_t*)calloc(P + 1, sizeof(size_t));
    int32_t* adj = (int32_t*)malloc((2 * ne + 1) * sizeof(int32_t));
    int32_t* queue = (int32_t*)malloc(P * sizeof(int32_t));
    int32_t* lab = (int32_t*)malloc(P * sizeof(int32_t));
    if (!off || !adj || !queue || !lab) {
        free(eu); free(ev); free(off); free(adj); free(queue); free(lab);
        return -2;
    }
    for (size_t e = 0; e < ne; ++e) { off[eu[e] + 1]++; off[ev[e] + 1]++; }
    for (size_t i = 0; i < P; ++i) off[i + 1] += off[i];
    {
        size_t* fill = (size_t*)malloc(P * sizeof(size_t));
        if (!fill) {
            free(eu); free(ev); free(off); free(adj); free(queue); free(lab);
            return -2;
        }
        memcpy(fill, off, P * sizeof(size_t));
        for (size_t e = 0; e < ne; ++e) {
            adj[fill[eu[e]]++] = ev[e];
            adj[fill[ev[e]]++] = eu[e];
        }
        free(fill);
    }
    free(eu); free(ev);

    /* Pass 2: breadth-first search from each unlabelled measurement in raster
     * order; the seed index is the label of everything it reaches. */
    for (size_t i = 0; i < P; ++i) lab[i] = -1;
    for (int32_t s = 0; s < (int32_t)P; ++s) {
        if (lab[s] != -1 || !is_measurement(range[s])) continue;
        size_t head = 0, tail = 0;
        lab[s] = s;
        queue[tail++] = s;
        while (head < tail) {
            const int32_t u = queue[head++];
            for (size_t j = off[u]; j < off[u + 1]; ++j) {
                const int32_t v = adj[j];
                if (lab[v] == -1) { lab[v] = s; queue[tail++] = v; }
            }
        }
    }
    memcpy(labels_out, lab, P * sizeof(int32_t));
    free(off); free(adj); free(queue); free(lab);
    return 0;
}

/* Section III.B.1: a labelled cluster with fewer than min_points measurements
 * is not a cluster candidate; its pixels become -1 like missing ones.  Plain
 * definition: one histogram pass over the canonical labels, one filter pass.
 * min_points == 0 leaves the labels as they are. */
int32_t flic_oracle_filter_small(const int32_t* labels, int32_t H, int32_t W,
                                 int32_t min_points, int32_t* labels_out) {
    if (!labels || !labels_out) return -1;
    if (H < 1 || W < 1 || min_points < 0) return -1;
    if ((int64_t)H * (int64_t)W > (int64_t)INT32_MAX) return -1;
    const size_t P = (size_t)H * (size_t)W;
    for (size_t i = 0; i < P; ++i)
        if (labels[i] < -1 || labels[i] >= (int64_t)P) return -1;
    int64_t* count = (int64_t*)calloc(P, sizeof(int64_t));
    if (!count) return -2;
    for (size_t i = 0; i < P; ++i)
        if (labels[i] >= 0) count[labels[i]] += 1;
    for (size_t i = 0; i < P; ++i) {
        const int32_t l = labels[i];
        labels_out[i] = (l >= 0 && count[l] >= min_points) ? l : -1;
    }
    free(count);
    return 0;
}

/* Section III.A, ground extraction, in the paper's order of steps.
 *   1. Eq. (2): for every pair of vertically adjacent measurements, the
 *      surface angle beta at the upper cell (range d1) between its beam and
 *      the surface it spans with the lower cell (range d2):
 *      tan(beta) = (d2 sin a) / (d1 - d2 cos a), sin a and cos a from the
 *      tables of the lower cell's row.
 *   2. The pair spans a horizontal surface when tan(beta) lies in the lower
 *      row's window [tan_lo, tan_hi] (tangents of the upper beam's angle
 *      below the horizontal -+ the threshold angle, from the caller).
 *   3. A cell is tested with the cell above it; the first row has no row
 *      above and takes the result of the second row's test (the paper
 *      extends beta_2 to the first channel), and so does any cell whose
 *      upper neighbour is missing: it takes its pair with the cell below.
 *   4. Height image: z = sensor_height + d sin(delta_r) over the wheel plane;
 *      a horizontal cell is ground only when z <= (d cos(delta_r)) tan_theta,
 *      the slope line from the wheel position.
 * Every float operation is one binary32 rounding (division included). */
static int pair_horizontal(const float* range, int32_t W, int32_t r,  /* rows r-1, r */
                           int32_t c, const float* sin_a, const float* cos_a,
                           const float* tan_lo, const float* tan_hi) {
    const float d1 = range[(size_t)(r - 1) * W + c];
    const float d2 = range[(size_t)r * W + c];
    if (!is_measurement(d1) || !is_measurement(d2)) return 0;
    const float num = d2 * sin_a[r];
    const float den = d1 - d2 * cos_a[r];
    const float tan_beta = num / den;
    return tan_lo[r] <= tan_beta && tan_beta <= tan_hi[r];
}

int32_t flic_oracle_ground(const float* range, int32_t H, int32_t W,
                           const float* sin_a, const float* cos_a,
                           const float* tan_lo, const float* tan_hi,
                           const float* sin_d, const float* cos_d,
                           float sensor_height, float tan_theta,
                           uint8_t* ground_out, float* range_out) {
    if (!range || !sin_a || !cos_a || !tan_lo || !tan_hi || !sin_d || !cos_d) return -1;
    if (!ground_out || !range_out) return -1;
    if (H < 1 || W < 1) return -1;
    if ((int64_t)H * (int64_t)W > (int64_t)INT32_MAX) return -1;
    for (int32_t r = 0; r < H; ++r) {
        for (int32_t c = 0; c < W; ++c) {
            const size_t i = (size_t)r * W + c;
            const float d = range[i];
            int ground = 0;
            if (is_measurement(d)) {
                int horizontal;
                if (r >= 1 && is_measurement(range[i - W]))
                    horizontal = pair_horizontal(range, W, r, c, sin_a, cos_a, tan_lo, tan_hi);
                else
                    horizontal = r + 1 < H && pair_horizontal(range, W, r + 1, c, sin_a, cos_a, tan_lo, tan_hi);
                if (horizontal) {
                    const float z = sensor_height + d * sin_d[r];
                    const float line = (d * cos_d[r]) * tan_theta;
                    ground = z <= line;
                }
            }
            ground_out[i] = (uint8_t)ground;
            range_out[i] = ground ? 0.0f : d;
        }
    }
    return 0;
}
