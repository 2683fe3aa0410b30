/*
 * sgm_oracle.h -- plain CPU oracle for the SGM stereo hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * shares no code, header, table or helper with it.
 *
 * Every function is single-threaded scalar C on host pointers.  All data is
 * row-major; volumes are [height][width][ndisp] with the disparity index
 * fastest.  Disparity maps are uint16 with 0xFFFF marking an invalid pixel.
 * The functions do not validate their arguments beyond what the caller
 * (oracle/__init__.py) already checks.
 */
#ifndef SGM_ORACLE_H
#define SGM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGM_ORACLE_INVALID 0xFFFFu

/* Census transform, Sec. 2.2.1 (zero margin outside the image) and
 * Sec. 2.3.1 (centre pixel omitted).  win_w x win_h window, both odd. */
void sgm_oracle_census(const uint8_t* img, int width, int height,
                       int win_w, int win_h, uint64_t* out);

/* Hamming matching cost, Eq. (image_matching) with Phi = Hamming distance of
 * census descriptors (Sec. 2.1.1); 255 where x - d < 0 (Sec. 2.3.1). */
void sgm_oracle_cost(const uint64_t* census_left, const uint64_t* census_right,
                     int width, int height, int ndisp, uint8_t* cost);

/* One step of Eq. (sgm_path) at one pixel: L_r(p, .) from the cost vector of p
 * and L_r(p - r, .) (`prev`, NULL at the first pixel of a path). */
void sgm_oracle_path_step(const uint8_t* cost_p, const uint16_t* prev, int ndisp,
                          int p1, int p2, uint16_t* cur);

/* One SGM path L_r of Eq. (sgm_path), normalised by the predecessor's minimum,
 * for the step r = (dx, dy): the predecessor of p is p - r. */
void sgm_oracle_path(const uint8_t* cost, int width, int height, int ndisp,
                     int dx, int dy, int p1, int p2, uint16_t* path_out);

/* Aggregated volume of Eq. (sgm_path_aggr) over the 4- or 8-path set. */
void sgm_oracle_aggregate(const uint8_t* cost, int width, int height, int ndisp,
                          int npaths, int p1, int p2, uint16_t* agg);

/* Aggregated costs at one pixel only: runs the line recursions that end at
 * (x, y) for every path of the set.  Used to check full-size outputs at
 * sampled pixels. */
void sgm_oracle_aggregate_at(const uint8_t* cost, int width, int height, int ndisp,
                             int npaths, int p1, int p2, int x, int y,
                             uint16_t* agg_px);

/* Winner-takes-all, Eq. (wta); ties go to the smallest disparity. */
void sgm_oracle_wta(const uint16_t* agg, int width, int height, int ndisp,
                    uint16_t* disp_left);

/* Approximate right disparity map, Eq. (right_disparity). */
void sgm_oracle_right_disparity(const uint16_t* agg, int width, int height,
                                int ndisp, uint16_t* disp_right);

/* Left-right consistency check, Eq. (LR_check) with tolerance t. */
void sgm_oracle_lr_check(const uint16_t* disp_left, const uint16_t* disp_right,
                         int width, int height, int tolerance, uint16_t* disp);

/* 3x3 median of the valid pixels (Sec. 2.1.3, Sec. 2.2.4, App. F). */
void sgm_oracle_median3x3(const uint16_t* disp, int width, int height,
                          uint16_t* out);

/* Median of nine values by the first five passes of a bubble-sort network
 * (App. F).  Exposed for the worked-example check. */
uint16_t sgm_oracle_median9(const uint16_t v[9]);

/* Index of the minimum by pairwise halving (App. D), n a power of two;
 * ties keep the lower index.  Exposed for the worked-example check. */
int sgm_oracle_map_reduce_argmin(const uint16_t* values, int n);

#ifdef __cplusplus
}
#endif
/* The whole path of oracle.run (census, cost, S_bar, D^L, D^R, LR check when
 * lr_tolerance >= 0, median when median3x3) with its independent work spread
 * over `nthreads` threads: the two census maps, rows of the cost volume and
 * of the per-pixel selection steps, and the lines of each path direction.
 * Same functions, same results; for timing the oracle on all host cores.
 * Returns 0, or -1 when memory runs out. */
int sgm_oracle_run_threaded(const uint8_t* left, const uint8_t* right, int width, int height,
                            int win_w, int win_h, int ndisp, int npaths, int p1, int p2,
                            int lr_tolerance, int median3x3, int nthreads,
                            uint16_t* disp_left, uint16_t* disp_right, uint16_t* disp);

/* Inverted, truncated NCC cost over win x win patches (win 5 or 9). */
void sgm_oracle_ncc_cost(const uint8_t* left, const uint8_t* right, int width, int height,
                         int win, int ndisp, uint8_t* cost);

#endif
