/*
 * sgm_oracle.c -- plain, slow, obviously correct CPU oracle for the SGM
 * stereo hot path of "ReS2tAC -- UAV-borne real-time SGM stereo optimized for
 * embedded ARM and CUDA devices" (Ruf et al., 2021).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  It shares no code
 * with the HIP kernels.
 *
 * Each function follows the paper's definition step by step, in its order and
 * notation.  Where the paper leaves a detail open, the reading taken is named
 * in the comment (the full list of readings lives with the design notes):
 *   census bit = [I(q) < I(p)], centre omitted, raster order dy-outer/dx-inner
 *   shifted in from the right, zero margin outside the image; cost 255 where
 *   x - d < 0; Gamma = {0..D-1}; every path value is reduced by the minimum of
 *   its predecessor; a path starts with L_r = C at its first pixel; missing
 *   d-1 / d+1 neighbours drop out; ties resolve to the smallest disparity;
 *   invalid = 0xFFFF; median pads with 0xFFFF and keeps invalid pixels invalid.
 */
#include "sgm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int inside(int x, int y, int width, int height) {
    return x >= 0 && x < width && y >= 0 && y < height;
}

/* Census transform (Sec. 2.2.1, Sec. 2.3.1).  For every neighbour q of p in the
 * win_w x win_h window, except p itself, one bit [I(q) < I(p)] is appended;
 * pixels outside the image read as zero (the zero-valued margin). */
void sgm_oracle_census(const uint8_t* img, int width, int height,
                       int win_w, int win_h, uint64_t* out) {
    const int rx = (win_w - 1) / 2;
    const int ry = (win_h - 1) / 2;
    for (int y = 0; y < height; ++y) {
        for (int x = 0; x < width; ++x) {
            const int centre = img[(size_t)y * width + x];
            uint64_t desc = 0;
            for (int dy = -ry; dy <= ry; ++dy) {
                for (int dx = -rx; dx <= rx; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const int qx = x + dx, qy = y + dy;
                    const int value = inside(qx, qy, width, height)
                                          ? img[(size_t)qy * width + qx] : 0;
                    desc = (desc << 1) | (uint64_t)(value < centre ? 1 : 0);
                }
            }
            out[(size_t)y * width + x] = desc;
        }
    }
}

static int popcount64(uint64_t v) {
    int n = 0;
    while (v) {
        n += (int)(v & 1u);
        v >>= 1;
    }
    return n;
}

/* Matching cost S(p, d) = Phi(I^L(px, py), I^R(px - d, py)), Eq. (image_matching),
 * with Phi the Hamming distance of the census descriptors (Sec. 2.1.1).  Where
 * the matching pixel px - d lies left of the image the cost is 0xFF
 * (Sec. 2.3.1). */
void sgm_oracle_cost(const uint64_t* census_left, const uint64_t* census_right,
                     int width, int height, int ndisp, uint8_t* cost) {
    for (int y = 0; y < height; ++y) {
        for (int x = 0; x < width; ++x) {
            for (int d = 0; d < ndisp; ++d) {
                int c = 255;
                if (x - d >= 0) {
                    c = popcount64(census_left[(size_t)y * width + x] ^
                                   census_right[(size_t)y * width + (x - d)]);
                }
                cost[((size_t)y * width + x) * ndisp + d] = (uint8_t)c;
            }
        }
    }
}

/* One step of Eq. (sgm_path):
 *   L_r(p, d) = S(p, d) + min_d' (L_r(p - r, d') + V(d, d')) - min_d' L_r(p - r, d')
 * with V = 0 (d' = d), P1 (|d - d'| = 1), P2 (|d - d'| > 1).  For P1 <= P2 the
 * minimum over d' equals min(L'(d), L'(d-1) + P1, L'(d+1) + P1, min L' + P2):
 * every d' with |d - d'| <= 1 also appears in the P2 term with a penalty no
 * smaller than its own.  `prev` is NULL at the first pixel of a path, where
 * L_r = S. */
void sgm_oracle_path_step(const uint8_t* cost_p, const uint16_t* prev, int ndisp,
                          int p1, int p2, uint16_t* cur) {
    if (prev == NULL) {
        for (int d = 0; d < ndisp; ++d) cur[d] = cost_p[d];
        return;
    }
    int min_prev = prev[0];
    for (int d = 1; d < ndisp; ++d)
        if (prev[d] < min_prev) min_prev = prev[d];
    for (int d = 0; d < ndisp; ++d) {
        int best = prev[d];
        if (d >= 1 && prev[d - 1] + p1 < best) best = prev[d - 1] + p1;
        if (d + 1 <= ndisp - 1 && prev[d + 1] + p1 < best) best = prev[d + 1] + p1;
        if (min_prev + p2 < best) best = min_prev + p2;
        cur[d] = (uint16_t)(cost_p[d] + best - min_prev);
    }
}

/* Path L_r for the step r = (dx, dy), with dx, dy in {-1, 0, 1}.  Pixels are
 * visited so that p - r always comes before p: rows in the order of dy, and
 * within a row columns in the order of dx. */
void sgm_oracle_path(const uint8_t* cost, int width, int height, int ndisp,
                     int dx, int dy, int p1, int p2, uint16_t* path_out) {
    for (int yi = 0; yi < height; ++yi) {
        const int y = (dy >= 0) ? yi : height - 1 - yi;
        for (int xi = 0; xi < width; ++xi) {
            const int x = (dx >= 0) ? xi : width - 1 - xi;
            const int px = x - dx, py = y - dy;
            const size_t idx = (size_t)y * width + x;
            const uint16_t* prev = NULL;
            if (inside(px, py, width, height))
                prev = path_out + ((size_t)py * width + px) * ndisp;
            sgm_oracle_path_step(cost + idx * ndisp, prev, ndisp, p1, p2,
                      path_out + idx * ndisp);
        }
    }
}

/* The path sets: the first four are the two horizontal and the two vertical
 * paths (4-path variant, Sec. 3.1.4); the eight-path set adds the diagonals. */
static const int kDirs[8][2] = {
    {1, 0}, {-1, 0}, {0, 1}, {0, -1},     /* LR, RL, TB, BT */
    {1, 1}, {-1, 1}, {1, -1}, {-1, -1},   /* TLBR, TRBL, BLTR, BRTL */
};

/* S_bar(p, d) = sum_r L_r(p, d), Eq. (sgm_path_aggr). */
void sgm_oracle_aggregate(const uint8_t* cost, int width, int height, int ndisp,
                          int npaths, int p1, int p2, uint16_t* agg) {
    const size_t n = (size_t)width * height * ndisp;
    uint32_t* sum = (uint32_t*)calloc(n, sizeof(uint32_t));
    uint16_t* path = (uint16_t*)malloc(n * sizeof(uint16_t));
    for (int r = 0; r < npaths; ++r) {
        sgm_oracle_path(cost, width, height, ndisp, kDirs[r][0], kDirs[r][1],
                        p1, p2, path);
        for (size_t i = 0; i < n; ++i) sum[i] += path[i];
    }
    for (size_t i = 0; i < n; ++i) agg[i] = (uint16_t)sum[i];
    free(path);
    free(sum);
}

/* S_bar at a single pixel: for each path, walk back from (x, y) along -r to
 * the first pixel of its line, then run Eq. (sgm_path) forward to (x, y). */
void sgm_oracle_aggregate_at(const uint8_t* cost, int width, int height, int ndisp,
                             int npaths, int p1, int p2, int x, int y,
                             uint16_t* agg_px) {
    uint16_t* a = (uint16_t*)malloc((size_t)ndisp * sizeof(uint16_t));
    uint16_t* b = (uint16_t*)malloc((size_t)ndisp * sizeof(uint16_t));
    uint32_t* sum = (uint32_t*)calloc((size_t)ndisp, sizeof(uint32_t));
    for (int r = 0; r < npaths; ++r) {
        const int dx = kDirs[r][0], dy = kDirs[r][1];
        int sx = x, sy = y;
        while (inside(sx - dx, sy - dy, width, height)) {
            sx -= dx;
            sy -= dy;
        }
        uint16_t* prev = NULL;
        uint16_t* cur = a;
        for (;;) {
            sgm_oracle_path_step(cost + ((size_t)sy * width + sx) * ndisp, prev, ndisp, p1, p2, cur);
            if (sx == x && sy == y) break;
            prev = cur;
            cur = (cur == a) ? b : a;
            sx += dx;
            sy += dy;
        }
        for (int d = 0; d < ndisp; ++d) sum[d] += cur[d];
    }
    for (int d = 0; d < ndisp; ++d) agg_px[d] = (uint16_t)sum[d];
    free(sum);
    free(b);
    free(a);
}

/* D(p) = argmin_d S_bar(p, d), Eq. (wta); the first (smallest) d wins ties. */
void sgm_oracle_wta(const uint16_t* agg, int width, int height, int ndisp,
                    uint16_t* disp_left) {
    for (size_t i = 0; i < (size_t)width * height; ++i) {
        const uint16_t* v = agg + i * ndisp;
        int best = 0;
        for (int d = 1; d < ndisp; ++d)
            if (v[d] < v[best]) best = d;
        disp_left[i] = (uint16_t)best;
    }
}

/* D^R(p) = argmin_d S_bar((px + d, py), d), Eq. (right_disparity), over the d
 * with px + d inside the image; the smallest d wins ties. */
void sgm_oracle_right_disparity(const uint16_t* agg, int width, int height,
                                int ndisp, uint16_t* disp_right) {
    for (int y = 0; y < height; ++y) {
        for (int x = 0; x < width; ++x) {
            int best = 0;
            uint16_t best_cost = agg[((size_t)y * width + x) * ndisp + 0];
            for (int d = 1; d < ndisp && x + d < width; ++d) {
                const uint16_t c = agg[((size_t)y * width + (x + d)) * ndisp + d];
                if (c < best_cost) {
                    best_cost = c;
                    best = d;
                }
            }
            disp_right[(size_t)y * width + x] = (uint16_t)best;
        }
    }
}

/* Eq. (LR_check): keep D^L(p) if |D^L(p) - D^R(px - D^L(p), py)| <= t, else
 * invalid; also invalid when px - D^L(p) falls left of the image. */
void sgm_oracle_lr_check(const uint16_t* disp_left, const uint16_t* disp_right,
                         int width, int height, int tolerance, uint16_t* disp) {
    for (int y = 0; y < height; ++y) {
        for (int x = 0; x < width; ++x) {
            const size_t i = (size_t)y * width + x;
            const int dl = disp_left[i];
            uint16_t out = SGM_ORACLE_INVALID;
            if (dl != (int)SGM_ORACLE_INVALID && x - dl >= 0) {
                const int dr = disp_right[(size_t)y * width + (x - dl)];
                const int diff = dl > dr ? dl - dr : dr - dl;
                if (diff <= tolerance) out = (uint16_t)dl;
            }
            disp[i] = out;
        }
    }
}

/* Median of nine wires: five bubble passes, each comparator moving the smaller
 * value to the upper wire (App. F).  Pass k carries the largest remaining value
 * down to wire 8 - k, so after five passes wires 4..8 hold the five largest
 * values in order and wire 4 holds the median. */
uint16_t sgm_oracle_median9(const uint16_t v_in[9]) {
    uint16_t v[9];
    memcpy(v, v_in, sizeof(v));
    for (int pass = 0; pass < 5; ++pass) {
        for (int i = 0; i + 1 <= 8 - pass; ++i) {
            if (v[i] > v[i + 1]) {
                const uint16_t t = v[i];
                v[i] = v[i + 1];
                v[i + 1] = t;
            }
        }
    }
    return v[4];
}

/* 3x3 median over pixels with a valid disparity (Sec. 2.1.3, Sec. 2.2.4).
 * Neighbours outside the image contribute 0xFFFF; invalid pixels stay
 * invalid. */
void sgm_oracle_median3x3(const uint16_t* disp, int width, int height,
                          uint16_t* out) {
    for (int y = 0; y < height; ++y) {
        for (int x = 0; x < width; ++x) {
            const size_t i = (size_t)y * width + x;
            if (disp[i] == SGM_ORACLE_INVALID) {
                out[i] = SGM_ORACLE_INVALID;
                continue;
            }
            uint16_t w[9];
            int k = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                    w[k++] = inside(x + dx, y + dy, width, height)
                                 ? disp[(size_t)(y + dy) * width + (x + dx)]
                                 : (uint16_t)SGM_ORACLE_INVALID;
            out[i] = sgm_oracle_median9(w);
        }
    }
}

/* Minimum search by pairwise halving (App. D): in each round element i is
 * compared with element i + n/2 and the smaller survives at i, together with
 * its label; log2(n) rounds.  Equal values keep the lower label. */
int sgm_oracle_map_reduce_argmin(const uint16_t* values, int n) {
    uint16_t* v = (uint16_t*)malloc((size_t)n * sizeof(uint16_t));
    int* label = (int*)malloc((size_t)n * sizeof(int));
    for (int i = 0; i < n; ++i) {
        v[i] = values[i];
        label[i] = i;
    }
    for (int half = n / 2; half >= 1; half /= 2) {
        for (int i = 0; i < half; ++i) {
            const int j = i + half;
            if (v[j] < v[i] || (v[j] == v[i] && label[j] < label[i])) {
                v[i] = v[j];
                label[i] = label[j];
            }
        }
    }
    const int best = label[0];
    free(label);
    free(v);
    return best;
}

/* Inverted, truncated normalised cross-correlation cost (Sec. 2.1.1,
 * Sec. 2.2.1): s = 1 - max(0, Phi_NCC) over a win x win patch, scaled to the
 * uint8 cost range as round(255 s).  Readings: pixels outside the image read
 * as zero (the same zero margin as the census window); a patch with zero
 * variance has no correlation (Phi = 0, cost 255); x - d < 0 costs 255.
 * Phi is formed from exact integer window sums,
 *   Phi = (n S_LR - S_L S_R) / (sqrt(n S_LL - S_L^2) * sqrt(n S_RR - S_R^2)),
 * then evaluated in float32 in exactly this order with IEEE operations:
 *   den = sqrtf(vL) * sqrtf(vR); phi = num / den; s = 1 - max(0, phi);
 *   cost = rint(255 * s) clamped to [0, 255] (ties to even). */
static int pixel_at(const uint8_t* img, int width, int height, int x, int y) {
    return inside(x, y, width, height) ? img[(size_t)y * width + x] : 0;
}

void sgm_oracle_ncc_cost(const uint8_t* left, const uint8_t* right, int width, int height,
                         int win, int ndisp, uint8_t* cost) {
    const int r = (win - 1) / 2;
    const int n = win * win;
    for (int y = 0; y < height; ++y) {
        for (int x = 0; x < width; ++x) {
            for (int d = 0; d < ndisp; ++d) {
                uint8_t c = 255;
                if (x - d >= 0) {
                    long sl = 0, sr = 0, sll = 0, srr = 0, slr = 0;
                    for (int dy = -r; dy <= r; ++dy) {
                        for (int dx = -r; dx <= r; ++dx) {
                            const long a = pixel_at(left, width, height, x + dx, y + dy);
                            const long b = pixel_at(right, width, height, x - d + dx, y + dy);
                            sl += a;
                            sr += b;
                            sll += a * a;
                            srr += b * b;
                            slr += a * b;
                        }
                    }
                    const long num = n * slr - sl * sr;
                    const long vl = n * sll - sl * sl;
                    const long vr = n * srr - sr * sr;
                    if (vl > 0 && vr > 0) {
                        const float den = sqrtf((float)vl) * sqrtf((float)vr);
                        const float phi = (float)num / den;
                        const float s = 1.0f - (phi > 0.0f ? phi : 0.0f);
                        float v = rintf(255.0f * s);
                        if (v < 0.0f) v = 0.0f;
                        if (v > 255.0f) v = 255.0f;
                        c = (uint8_t)v;
                    }
                }
                cost[((size_t)y * width + x) * ndisp + d] = c;
            }
        }
    }
}
