/*
 * FP64 reference ("oracle") for the multi-scale hierarchical block matching hot
 * path.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
 * leg of the benchmark call it; the product library never links, loads or calls
 * it, and the two share no code.
 *
 * Every function below is the plain definition written out with direct loops in
 * double precision: no running sums, no blocking, no reuse across candidates.
 * Where the paper is silent or garbled, the adopted reading is stated at the
 * function and listed with the others in the design notes.
 *
 * Conventions shared by all functions
 *   - images are row-major double arrays, H rows by W columns, no padding;
 *   - window reads clamp to the nearest edge pixel (replicate border);
 *   - the right-image column of candidate z for left column j is j - z
 *     (left-reference convention for rectified pairs);
 *   - candidate z is valid iff 0 <= z <= min(D_k - 1, j).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Threads of the OpenMP loops below (for timing the oracle on one core). */
void omp_set_num_threads(int);
void orc_set_threads(int n) { omp_set_num_threads(n < 1 ? 1 : n); }

/* One Gaussian-pyramid step (Section III, K-level Gaussian pyramid).  The paper
 * does not name the blur; the reading is the 5-tap binomial [1 4 6 4 1]/16 in
 * each direction, sampled at even positions, output size ceil(H/2) x ceil(W/2),
 * written here as the full 25-tap 2-D sum. */
void orc_reduce(const double* in, int H, int W, double* out)
{
    static const double w[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
    const int Ho = (H + 1) / 2, Wo = (W + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < Ho; ++y) {
        for (int x = 0; x < Wo; ++x) {
            double s = 0.0;
            for (int a = -2; a <= 2; ++a)
                for (int b = -2; b <= 2; ++b)
                    s += w[a + 2] * w[b + 2] *
                         in[(size_t)clampi(2 * y + a, 0, H - 1) * W + clampi(2 * x + b, 0, W - 1)];
            out[(size_t)y * Wo + x] = s;
        }
    }
}

/* The adjoint (transpose) of orc_reduce, for carrying an image gradient from a
 * pyramid level to the level below: every coarse value is scattered with its
 * 25 binomial weights onto the clamped fine positions its reduce read from.
 * out (H x W) is overwritten. */
void orc_reduce_adjoint(const double* G, int H, int W, double* out)
{
    static const double w[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
    const int Ho = (H + 1) / 2, Wo = (W + 1) / 2;
    memset(out, 0, sizeof(double) * (size_t)H * W);
    for (int y = 0; y < Ho; ++y)
        for (int x = 0; x < Wo; ++x)
            for (int a = -2; a <= 2; ++a)
                for (int b = -2; b <= 2; ++b)
                    out[(size_t)clampi(2 * y + a, 0, H - 1) * W + clampi(2 * x + b, 0, W - 1)] +=
                        w[a + 2] * w[b + 2] * G[(size_t)y * Wo + x];
}

/* The same 5x5 binomial blur at every pixel: Section IV blurs the input image
 * before matching (matching on a blurred level 0 is the pre-blur variant):
 * out(y, x) = sum_{a,b} w_a w_b in(clamp(y + a), clamp(x + b)). */
void orc_blur(const double* in, int H, int W, double* out)
{
    static const double w[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            double s = 0.0;
            for (int a = -2; a <= 2; ++a)
                for (int b = -2; b <= 2; ++b)
                    s += w[a + 2] * w[b + 2] * in[(size_t)clampi(y + a, 0, H - 1) * W + clampi(x + b, 0, W - 1)];
            out[(size_t)y * W + x] = s;
        }
    }
}

/* Zero-mean normalised cross-correlation of the (2n+1)^2 window of L centred at
 * (i, j) and the window of R centred at (i, j - z) (Eq. 2, with the matching
 * cost of Eq. 1).  Readings: each view is centred by its own window mean and the
 * normaliser is the product of the two window standard deviations, so the value
 * is C / sqrt(A B) with A, B, C the centred sums of squares and cross products.
 * A window is flat when its variance A / N is at most `eps`; a flat window scores
 * 0.  The result is clamped to [-1, 1] against rounding. */
double orc_zncc(const double* L, const double* R, int H, int W, int n,
                int i, int j, int z, double eps)
{
    const int N = (2 * n + 1) * (2 * n + 1);
    double sl = 0.0, sr = 0.0;
    for (int a = -n; a <= n; ++a)
        for (int b = -n; b <= n; ++b) {
            const int y = clampi(i + a, 0, H - 1);
            sl += L[(size_t)y * W + clampi(j + b, 0, W - 1)];
            sr += R[(size_t)y * W + clampi(j - z + b, 0, W - 1)];
        }
    const double ml = sl / N, mr = sr / N;
    double A = 0.0, B = 0.0, C = 0.0;
    for (int a = -n; a <= n; ++a)
        for (int b = -n; b <= n; ++b) {
            const int y = clampi(i + a, 0, H - 1);
            const double l = L[(size_t)y * W + clampi(j + b, 0, W - 1)] - ml;
            const double r = R[(size_t)y * W + clampi(j - z + b, 0, W - 1)] - mr;
            A += l * l;
            B += r * r;
            C += l * r;
        }
    if (A <= N * eps || B <= N * eps) return 0.0;
    double rho = C / sqrt(A * B);
    if (rho > 1.0) rho = 1.0;
    if (rho < -1.0) rho = -1.0;
    return rho;
}

/* Candidate interval of pixel (i, j) at one level.
 * Full search (coarse == NULL, Eqs. 3-4): [0, min(D_k - 1, j)].
 * Restricted search (Eqs. 8-9, first branch): the prior is the coarser map
 * upsampled by nearest neighbour with its values doubled,
 * dhat = 2 d^{k+1}(i/2, j/2); with c = min(dhat, j) the interval is
 * [max(0, c - r), min(D_k - 1, j, c + r)].  Readings: the paper's interval
 * around dhat, stated as open and as three candidates, is taken as the closed
 * radius-r interval, and the prior is doubled because d_max halves per level. */
static void cand_range(int i, int j, int Dk, const int16_t* coarse, int Wc,
                       int r, int* lo, int* hi)
{
    int top = Dk - 1 < j ? Dk - 1 : j;
    if (!coarse) {
        *lo = 0;
        *hi = top;
        return;
    }
    int dh = 2 * (int)coarse[(size_t)(i / 2) * Wc + (j / 2)];
    int c = dh < j ? dh : j;
    *lo = c - r > 0 ? c - r : 0;
    *hi = c + r < top ? c + r : top;
}

/* Winner-take-all matching of one level (Eqs. 3-4 for a full search, Eqs. 8-9
 * first branch for a restricted one).  Outputs per pixel: d = the lowest valid z
 * whose score is maximal (ties break to the lowest z), C = that score, and C2 =
 * the second-largest score among the valid candidates (-inf when there is only
 * one), so tests can tell genuine near-ties apart. */
void orc_match_level(const double* L, const double* R, int H, int W, int n, int Dk,
                     const int16_t* coarse, int Hc, int Wc, int r, double eps,
                     int16_t* d, double* C, double* C2)
{
    (void)Hc;
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            int lo, hi;
            cand_range(i, j, Dk, coarse, Wc, r, &lo, &hi);
            double best = -INFINITY, second = -INFINITY;
            int bz = lo;
            for (int z = lo; z <= hi; ++z) {
                const double rho = orc_zncc(L, R, H, W, n, i, j, z, eps);
                if (rho > best) {
                    second = best;
                    best = rho;
                    bz = z;
                } else if (rho > second) {
                    second = rho;
                }
            }
            d[(size_t)i * W + j] = (int16_t)bz;
            C[(size_t)i * W + j] = best;
            C2[(size_t)i * W + j] = second;
        }
    }
}

/* Soft-argmax at the finest level (an addition to the paper: the differentiable
 * form).  Candidates are the restricted interval of radius rs around the doubled
 * level-1 prior; p_z = exp((rho_z - max rho) / tau) / sum, d_soft = sum p_z z.
 * The hard winner-take-all over the same interval is returned too. */
void orc_soft_level0(const double* L, const double* R, int H, int W, int n, int D,
                     const int16_t* coarse, int Hc, int Wc, int rs, double tau, double eps,
                     double* dsoft, int16_t* dhard, double* C, double* C2)
{
    (void)Hc;
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < H; ++i) {
        double rho[1024];
        for (int j = 0; j < W; ++j) {
            int lo, hi;
            cand_range(i, j, D, coarse, Wc, rs, &lo, &hi);
            double best = -INFINITY, second = -INFINITY;
            int bz = lo;
            for (int z = lo; z <= hi; ++z) {
                rho[z - lo] = orc_zncc(L, R, H, W, n, i, j, z, eps);
                if (rho[z - lo] > best) {
                    second = best;
                    best = rho[z - lo];
                    bz = z;
                } else if (rho[z - lo] > second) {
                    second = rho[z - lo];
                }
            }
            double sp = 0.0, spz = 0.0;
            for (int z = lo; z <= hi; ++z) {
                const double p = exp((rho[z - lo] - best) / tau);
                sp += p;
                spz += p * z;
            }
            dsoft[(size_t)i * W + j] = spz / sp;
            dhard[(size_t)i * W + j] = (int16_t)bz;
            C[(size_t)i * W + j] = best;
            C2[(size_t)i * W + j] = second;
        }
    }
}

/* Gradient of sum_{ij} gd(i,j) d_soft(i,j) with respect to every pixel of L and
 * R, with the level-1 prior held fixed (it is piecewise constant in the inputs).
 *   dd/drho_z = p_z (z - d_soft) / tau;
 *   drho/dl_ab = (r_ab - mu_r)/sqrt(AB) - rho (l_ab - mu_l)/A;
 *   drho/dr_ab = (l_ab - mu_l)/sqrt(AB) - rho (r_ab - mu_r)/B;
 * flat candidates (score fixed at 0) contribute nothing; a clamped read passes
 * its gradient to the edge pixel it read.  Only source pixels with rows in
 * [i0, i1) contribute (i0 = 0, i1 = H for the whole image).  Serial on purpose:
 * the scatter is written as the plain sum. */
void orc_backward(const double* L, const double* R, int H, int W, int n, int D,
                  const int16_t* coarse, int Hc, int Wc, int rs, double tau, double eps,
                  const double* gd, int i0, int i1, double* gL, double* gR)
{
    (void)Hc;
    const int N = (2 * n + 1) * (2 * n + 1);
    memset(gL, 0, sizeof(double) * (size_t)H * W);
    memset(gR, 0, sizeof(double) * (size_t)H * W);
    double rho[1024], ml[1024], mr[1024], A[1024], B[1024], Cc[1024];
    int flat[1024];
    for (int i = i0; i < i1; ++i) {
        for (int j = 0; j < W; ++j) {
            const double g = gd[(size_t)i * W + j];
            if (g == 0.0) continue;
            int lo, hi;
            cand_range(i, j, D, coarse, Wc, rs, &lo, &hi);
            double best = -INFINITY;
            for (int z = lo; z <= hi; ++z) {
                const int q = z - lo;
                double sl = 0.0, sr = 0.0;
                for (int a = -n; a <= n; ++a)
                    for (int b = -n; b <= n; ++b) {
                        const int y = clampi(i + a, 0, H - 1);
                        sl += L[(size_t)y * W + clampi(j + b, 0, W - 1)];
                        sr += R[(size_t)y * W + clampi(j - z + b, 0, W - 1)];
                    }
                ml[q] = sl / N;
                mr[q] = sr / N;
                A[q] = B[q] = Cc[q] = 0.0;
                for (int a = -n; a <= n; ++a)
                    for (int b = -n; b <= n; ++b) {
                        const int y = clampi(i + a, 0, H - 1);
                        const double l = L[(size_t)y * W + clampi(j + b, 0, W - 1)] - ml[q];
                        const double r = R[(size_t)y * W + clampi(j - z + b, 0, W - 1)] - mr[q];
                        A[q] += l * l;
                        B[q] += r * r;
                        Cc[q] += l * r;
                    }
                flat[q] = (A[q] <= N * eps || B[q] <= N * eps);
                if (flat[q]) {
                    rho[q] = 0.0;
                } else {
                    rho[q] = Cc[q] / sqrt(A[q] * B[q]);
                    if (rho[q] > 1.0) rho[q] = 1.0;
                    if (rho[q] < -1.0) rho[q] = -1.0;
                }
                if (rho[q] > best) best = rho[q];
            }
            double sp = 0.0, spz = 0.0;
            double p[1024];
            for (int z = lo; z <= hi; ++z) {
                p[z - lo] = exp((rho[z - lo] - best) / tau);
                sp += p[z - lo];
                spz += p[z - lo] * z;
            }
            const double ds = spz / sp;
            for (int z = lo; z <= hi; ++z) {
                const int q = z - lo;
                if (flat[q]) continue;
                const double gz = g * (p[q] / sp) * (z - ds) / tau;
                const double s = sqrt(A[q] * B[q]);
                const double rr = Cc[q] / s;
                for (int a = -n; a <= n; ++a)
                    for (int b = -n; b <= n; ++b) {
                        const int y = clampi(i + a, 0, H - 1);
                        const size_t il = (size_t)y * W + clampi(j + b, 0, W - 1);
                        const size_t ir = (size_t)y * W + clampi(j - z + b, 0, W - 1);
                        const double l = L[il] - ml[q];
                        const double r = R[ir] - mr[q];
                        gL[il] += gz * (r / s - rr * l / A[q]);
                        gR[ir] += gz * (l / s - rr * r / B[q]);
                    }
            }
        }
    }
}

/* Scores at a list of (i, j, z) triples (Eq. 2), for sampled comparisons. */
void orc_zncc_many(const double* L, const double* R, int H, int W, int n, double eps,
                   const int32_t* ii, const int32_t* jj, const int32_t* zz, int count, double* out)
{
#pragma omp parallel for schedule(static)
    for (int q = 0; q < count; ++q) out[q] = orc_zncc(L, R, H, W, n, ii[q], jj[q], zz[q], eps);
}

/* orc_match_level restricted to a list of pixels (same outputs, one per pixel). */
void orc_match_pixels(const double* L, const double* R, int H, int W, int n, int Dk,
                      const int16_t* coarse, int Hc, int Wc, int r, double eps,
                      const int32_t* ii, const int32_t* jj, int count,
                      int16_t* d, double* C, double* C2)
{
    (void)Hc;
#pragma omp parallel for schedule(dynamic, 8)
    for (int q = 0; q < count; ++q) {
        const int i = ii[q], j = jj[q];
        int lo, hi;
        cand_range(i, j, Dk, coarse, Wc, r, &lo, &hi);
        double best = -INFINITY, second = -INFINITY;
        int bz = lo;
        for (int z = lo; z <= hi; ++z) {
            const double rho = orc_zncc(L, R, H, W, n, i, j, z, eps);
            if (rho > best) {
                second = best;
                best = rho;
                bz = z;
            } else if (rho > second) {
                second = rho;
            }
        }
        d[q] = (int16_t)bz;
        C[q] = best;
        C2[q] = second;
    }
}

/* Selective median filtering (Section III.D, Eq. 10).  A pixel whose matched
 * cost is good (C > alpha) keeps its disparity; any other pixel takes the median
 * of the disparities of the good pixels of the 5x5 patch around it.  Readings:
 * the patch holds only pixels inside the image; the median of an even count is
 * the lower one; with no good pixel in the patch the disparity is kept; every
 * pixel reads the unfiltered map (d_in), so the order of the pixels does not
 * matter.  Values are sorted by insertion, the plainest correct way. */
void orc_median(const int16_t* d_in, const double* C, int H, int W, double alpha, int16_t* d_out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            const size_t o = (size_t)i * W + j;
            d_out[o] = d_in[o];
            if (C[o] > alpha) continue;
            int v[25], m = 0;
            for (int a = -2; a <= 2; ++a)
                for (int b = -2; b <= 2; ++b) {
                    const int y = i + a, x = j + b;
                    if (y < 0 || y >= H || x < 0 || x >= W) continue;
                    const size_t q = (size_t)y * W + x;
                    if (!(C[q] > alpha)) continue;
                    int t = m++;
                    while (t > 0 && v[t - 1] > d_in[q]) {
                        v[t] = v[t - 1];
                        --t;
                    }
                    v[t] = d_in[q];
                }
            if (m > 0) d_out[o] = (int16_t)v[(m - 1) / 2];
        }
    }
}

/* Keys' cubic convolution kernel with parameter a; a = -1/2 is the classical
 * bicubic interpolant, which reproduces polynomials up to degree two. */
static double keys_cubic(double x, double a)
{
    x = fabs(x);
    if (x <= 1.0) return (a + 2.0) * x * x * x - (a + 3.0) * x * x + 1.0;
    if (x < 2.0) return a * x * x * x - 5.0 * a * x * x + 8.0 * a * x - 4.0 * a;
    return 0.0;
}

/* Bicubic doubling of a coarse cost map (Section III.C: the cost map is carried
 * to the next finer level by bicubic interpolation).  Readings: the scale is
 * exactly 2 with pixel centres aligned, so fine pixel (i, j) sits at the coarse
 * position u = (i + 1/2)/2 - 1/2, v = (j + 1/2)/2 - 1/2; the kernel is Keys'
 * cubic with parameter a (a = -1/2 for the method); taps clamp to the nearest
 * edge sample.  Written as the full 16-tap sum.  Output H x W, the finer level
 * (H <= 2 Hc, W <= 2 Wc). */
void orc_bicubic_up(const double* Cc, int Hc, int Wc, int H, int W, double a, double* out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i) {
        const double u = (i + 0.5) / 2.0 - 0.5;
        const int i0 = (int)floor(u);
        for (int j = 0; j < W; ++j) {
            const double v = (j + 0.5) / 2.0 - 0.5;
            const int j0 = (int)floor(v);
            double s = 0.0;
            for (int m = i0 - 1; m <= i0 + 2; ++m)
                for (int q = j0 - 1; q <= j0 + 2; ++q)
                    s += keys_cubic(u - m, a) * keys_cubic(v - q, a) *
                         Cc[(size_t)clampi(m, 0, Hc - 1) * Wc + clampi(q, 0, Wc - 1)];
            out[(size_t)i * W + j] = s;
        }
    }
}

/* Confidence-gated matching of a finer level (Eqs. 8-9).  With the coarser map
 * d^{k+1} and its cost C^{k+1}: where the upsampled cost C^ = bicubic(C^{k+1})
 * exceeds beta, the search is restricted to the radius-r interval around the
 * doubled nearest-neighbour prior (first branch, the same interval as
 * orc_match_level); elsewhere it covers the full interval [0, min(D_k - 1, j)]
 * (second branch).  Outputs d', C', C2 as orc_match_level, plus full[p] = 1
 * where the second branch was taken. */
void orc_match_gated(const double* L, const double* R, int H, int W, int n, int Dk,
                     const int16_t* coarse, const double* coarse_cost, int Hc, int Wc, int r,
                     double beta, double eps, int16_t* d, double* C, double* C2, uint8_t* full)
{
    double* up = (double*)malloc(sizeof(double) * (size_t)H * W);
    orc_bicubic_up(coarse_cost, Hc, Wc, H, W, -0.5, up);
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            const size_t o = (size_t)i * W + j;
            const int restricted = up[o] > beta;
            int lo, hi;
            cand_range(i, j, Dk, restricted ? coarse : NULL, Wc, r, &lo, &hi);
            double best = -INFINITY, second = -INFINITY;
            int bz = lo;
            for (int z = lo; z <= hi; ++z) {
                const double rho = orc_zncc(L, R, H, W, n, i, j, z, eps);
                if (rho > best) {
                    second = best;
                    best = rho;
                    bz = z;
                } else if (rho > second) {
                    second = rho;
                }
            }
            d[o] = (int16_t)bz;
            C[o] = best;
            C2[o] = second;
            full[o] = (uint8_t)!restricted;
        }
    }
    free(up);
}

/* The neighbourhood-averaged score of pixel (i, j) at candidate z (Eq. 5, read
 * as a mean): the scores at z of the pixels of the 5x5 box around (i, j) that
 * lie inside the image and have z among their own candidates (z <= q for
 * column q), divided by their number. */
double orc_avg_score(const double* L, const double* R, int H, int W, int n, int i, int j, int z, double eps)
{
    double s = 0.0;
    int cnt = 0;
    for (int m = i - 2; m <= i + 2; ++m)
        for (int q = j - 2; q <= j + 2; ++q) {
            if (m < 0 || m >= H || q < 0 || q >= W || z > q) continue;
            s += orc_zncc(L, R, H, W, n, m, q, z, eps);
            ++cnt;
        }
    return s / cnt;
}

/* Disparity refinement by the neighbourhood-averaged disparity search image
 * (Eqs. 5-7).  A pixel whose matched cost C' is at most alpha takes the z that
 * maximises E^(z) = orc_avg_score over its own full interval
 * [0, min(D_k - 1, j)] (a reading: Eq. 6 names d_max, and this level's range is
 * D_k), and C = max E^; other pixels keep d' and C'.  Readings: the
 * neighbourhood is the 5x5 box of the median step; ties go to the lowest z.  C2
 * is the second-largest E^ of a re-picked pixel (-inf otherwise). */
static void aggregate_pixel(const double* L, const double* R, int H, int W, int n, int Dk,
                            const int16_t* d_in, const double* C_in, double alpha, double eps, int i, int j,
                            int16_t* d, double* C, double* C2)
{
    const size_t o = (size_t)i * W + j;
    *d = d_in[o];
    *C = C_in[o];
    *C2 = -INFINITY;
    if (C_in[o] > alpha) return;
    const int top = Dk - 1 < j ? Dk - 1 : j;
    double best = -INFINITY, second = -INFINITY;
    int bz = 0;
    for (int z = 0; z <= top; ++z) {
        const double e = orc_avg_score(L, R, H, W, n, i, j, z, eps);
        if (e > best) {
            second = best;
            best = e;
            bz = z;
        } else if (e > second) {
            second = e;
        }
    }
    *d = (int16_t)bz;
    *C = best;
    *C2 = second;
}

void orc_aggregate(const double* L, const double* R, int H, int W, int n, int Dk,
                   const int16_t* d_in, const double* C_in, double alpha, double eps,
                   int16_t* d, double* C, double* C2)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            const size_t o = (size_t)i * W + j;
            aggregate_pixel(L, R, H, W, n, Dk, d_in, C_in, alpha, eps, i, j, d + o, C + o, C2 + o);
        }
}

/* orc_aggregate restricted to a list of pixels (one output per pixel). */
void orc_aggregate_pixels(const double* L, const double* R, int H, int W, int n, int Dk,
                          const int16_t* d_in, const double* C_in, double alpha, double eps,
                          const int32_t* ii, const int32_t* jj, int count, int16_t* d, double* C, double* C2)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < count; ++q)
        aggregate_pixel(L, R, H, W, n, Dk, d_in, C_in, alpha, eps, ii[q], jj[q], d + q, C + q, C2 + q);
}

/* orc_avg_score at a list of (i, j, z) triples. */
void orc_avg_score_many(const double* L, const double* R, int H, int W, int n, double eps,
                        const int32_t* ii, const int32_t* jj, const int32_t* zz, int count, double* out)
{
#pragma omp parallel for schedule(static)
    for (int q = 0; q < count; ++q) out[q] = orc_avg_score(L, R, H, W, n, ii[q], jj[q], zz[q], eps);
}
