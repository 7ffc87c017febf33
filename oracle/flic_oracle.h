/*
 * flic_oracle.h -- CPU oracle for FLIC range-image clustering.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct statement of what the clustering computes; it exists so that tests
 * and the benchmark's CPU baseline can check the GPU library against it.  No
 * product code may link, load or call it, and it shares no code with the GPU
 * path.
 *
 * Semantics (FLIC, Hasecke, Hahn, Kummert, arXiv 2003.00575):
 *   - A pixel is a measurement iff its range is > 0 and finite (Section
 *     III.A: zero marks a missing / removed value).
 *   - Two pixels are connected when the squared Euclidean distance recovered
 *     by the cosine law, Eq. (4) D^2 = d1*d1 + d2*d2 - (2 cos a) * d1 * d2,
 *     is <= T^2 (Section III.B, one physical threshold T).
 *   - Neighbours: the same column k rows down, or the same row k columns to
 *     the right with 360-degree wrap, for k = 1..N (k = 1 is the direct
 *     4-neighbourhood of Section III.B.1; k >= 2 are the map/skip connections
 *     of Section III.B.2, taken densely).
 *   - Output: each measurement gets the smallest linear index r*W + c of its
 *     connected component; missing pixels get -1.
 *   - Ground extraction before clustering (Section III.A): cells on a near
 *     horizontal surface below a slope line are removed (range 0).
 *   - Optional cluster-size threshold (Section III.B.1, 100 points in the
 *     paper): components with fewer measurements are relabelled -1.
 */
#ifndef FLIC_ORACLE_H
#define FLIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Eq. (4) evaluated in IEEE binary32, each operation rounded to nearest-even:
 *   (d1*d1 + d2*d2) - ((2*cos_alpha) * (d1*d2))                            */
float flic_oracle_dist2(float d1, float d2, float cos_alpha);

/* Cluster one range image.
 *   range      host [H][W] row-major float32 metres
 *   cos_v      host [N][H]; cos_v[(k-1)*H + r] = cos(angle rows r, r+k);
 *              entries r >= H-k are never read
 *   cos_h      host [N][W]; cos_h[(k-1)*W + c] = cos(angle cols c, (c+k)%W)
 *   threshold  metres, finite and >= 0; the test is D^2 <= fl32(T*T)
 *   skip_depth N, 1 <= N <= 8, 2N < W
 *   labels_out host [H][W] int32, written only on success
 * Returns 0 on success, -1 for invalid arguments, -2 when memory runs out. */
int32_t flic_oracle_cluster(const float* range, int32_t H, int32_t W,
                            const float* cos_v, const float* cos_h,
                            float threshold, int32_t skip_depth,
                            int32_t* labels_out);

/* The same with the choice of skip edges: maps == 0 gives the dense skip
 * connections above (every pixel, offsets 2..N); maps == 1 the paper's Map
 * Connections (Section III.B.2): for each stride k = 2..N, only pixels whose
 * row and column are multiples of k connect to their k-th neighbour to the
 * right (with wrap) and below.  Direct (k = 1) edges are the same in both. */
int32_t flic_oracle_cluster_maps(const float* range, int32_t H, int32_t W,
                                 const float* cos_v, const float* cos_h,
                                 float threshold, int32_t skip_depth, int32_t maps,
                                 int32_t* labels_out);

/* Cluster-size threshold (Section III.B.1): every pixel whose label occurs
 * fewer than min_points times in `labels` becomes -1; others keep their
 * label.  labels is host [H][W] int32 with entries -1 or in [0, H*W);
 * labels_out may equal labels.  min_points >= 0 (0 and 1 keep every label).
 * Returns 0, -1 for invalid arguments, -2 when memory runs out.            */
int32_t flic_oracle_filter_small(const int32_t* labels, int32_t H, int32_t W,
                                 int32_t min_points, int32_t* labels_out);

/* Ground extraction (Section III.A, Eq. 1/2, the height image and the
 * first-channel rule).  A cell is tested with the cell above it, or, when it
 * is in the first row or the cell above is missing, takes the test of its
 * pair with the cell below.  Host arrays; per-row tables of H entries:
 *   sin_a, cos_a  sin / cos of the angle between rows r-1 and r (entry 0 unused)
 *   tan_lo, tan_hi  window of tan(beta) for the pair (r-1, r) to span a
 *                   horizontal surface (entry 0 unused)
 *   sin_d, cos_d  sin / cos of row r's elevation angle
 *   sensor_height metres of the sensor above the wheel plane
 *   tan_theta     slope of the height line (tan 10 degrees in the paper)
 * ground_out [H][W] gets 1 for a ground cell, else 0; range_out [H][W] is the
 * range with ground cells set to 0 (removed) and every other value copied.
 * Returns 0, -1 for invalid arguments, -2 when memory runs out.            */
int32_t flic_oracle_ground(const float* range, int32_t H, int32_t W,
                           const float* sin_a, const float* cos_a,
                           const float* tan_lo, const float* tan_hi,
                           const float* sin_d, const float* cos_d,
                           float sensor_height, float tan_theta,
                           uint8_t* ground_out, float* range_out);

#ifdef __cplusplus
}
#endif
#endif
