/*
 * sgm_oracle_mt.c -- the oracle's whole path with its independent work spread
 * over POSIX threads, for timing the oracle on every host core.
 *
 * TEST INFRASTRUCTURE ONLY (like sgm_oracle.c, whose functions it calls).  It
 * adds no arithmetic of its own: each stage calls the oracle's functions on
 * parts of the frame that do not depend on each other, and the results equal
 * oracle.run bit for bit (the CPU tests check this).
 *   census     the two images on two threads;
 *   cost       bands of rows (a pixel's costs need only its own row);
 *   S_bar      one direction at a time: the direction's lines -- each starts
 *              at a pixel whose predecessor p - r lies outside the image --
 *              are walked in parallel with the oracle's step function, then
 *              the path is added to the sum in bands of pixels;
 *   D^L, D^R,  bands of rows (Eq. wta, Eq. right_disparity and Eq. LR_check
 *   LR check   look at one row only);
 *   median     one thread (it is cheap).
 */
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#include "sgm_oracle.h"

typedef struct {
    void (*fn)(void* ctx, long begin, long end);
    void* ctx;
    long begin, end;
} Task;

static void* task_main(void* arg) {
    Task* t = (Task*)arg;
    t->fn(t->ctx, t->begin, t->end);
    return NULL;
}

/* fn(ctx, b, e) over [0, n) split into nthreads contiguous ranges. */
static void parallel_for(int nthreads, long n, void (*fn)(void*, long, long), void* ctx) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n) nthreads = n > 0 ? (int)n : 1;
    pthread_t th[256];
    Task task[256];
    if (nthreads > 256) nthreads = 256;
    for (int i = 0; i < nthreads; ++i) {
        task[i].fn = fn;
        task[i].ctx = ctx;
        task[i].begin = n * i / nthreads;
        task[i].end = n * (i + 1) / nthreads;
    }
    int started = 0;
    for (int i = 1; i < nthreads; ++i) {
        if (pthread_create(&th[i], NULL, task_main, &task[i]) != 0) break;
        started = i;
    }
    /* ranges whose thread could not start run here */
    task_main(&task[0]);
    for (int i = started + 1; i < nthreads; ++i) task_main(&task[i]);
    for (int i = 1; i <= started; ++i) pthread_join(th[i], NULL);
}

typedef struct {
    const uint8_t *left, *right;
    int width, height, win_w, win_h, ndisp, p1, p2, dx, dy, tolerance;
    uint64_t *cl, *cr;
    uint8_t* cost;
    uint16_t* path;
    uint32_t* sum;
    uint16_t *agg, *dl, *dr, *chk;
    int* starts;            /* (x, y) of every line start of the current direction */
} Ctx;

static void census_part(void* p, long b, long e) {
    Ctx* c = (Ctx*)p;
    for (long i = b; i < e; ++i)
        sgm_oracle_census(i == 0 ? c->left : c->right, c->width, c->height, c->win_w, c->win_h,
                          i == 0 ? c->cl : c->cr);
}

static void cost_rows(void* p, long b, long e) {
    Ctx* c = (Ctx*)p;
    const size_t w = (size_t)c->width;
    sgm_oracle_cost(c->cl + b * w, c->cr + b * w, c->width, (int)(e - b), c->ndisp,
                    c->cost + b * w * c->ndisp);
}

static int inside(int x, int y, int width, int height) {
    return x >= 0 && x < width && y >= 0 && y < height;
}

static void path_lines(void* p, long b, long e) {
    Ctx* c = (Ctx*)p;
    const size_t nd = (size_t)c->ndisp;
    for (long i = b; i < e; ++i) {
        int x = c->starts[2 * i], y = c->starts[2 * i + 1];
        const uint16_t* prev = NULL;
        while (inside(x, y, c->width, c->height)) {
            const size_t idx = (size_t)y * c->width + x;
            sgm_oracle_path_step(c->cost + idx * nd, prev, c->ndisp, c->p1, c->p2, c->path + idx * nd);
            prev = c->path + idx * nd;
            x += c->dx;
            y += c->dy;
        }
    }
}

static void add_path(void* p, long b, long e) {
    Ctx* c = (Ctx*)p;
    for (long i = b; i < e; ++i) c->sum[i] += c->path[i];
}

static void narrow_sum(void* p, long b, long e) {
    Ctx* c = (Ctx*)p;
    for (long i = b; i < e; ++i) c->agg[i] = (uint16_t)c->sum[i];
}

static void select_rows(void* p, long b, long e) {
    Ctx* c = (Ctx*)p;
    const size_t w = (size_t)c->width;
    const int rows = (int)(e - b);
    sgm_oracle_wta(c->agg + b * w * c->ndisp, c->width, rows, c->ndisp, c->dl + b * w);
    sgm_oracle_right_disparity(c->agg + b * w * c->ndisp, c->width, rows, c->ndisp, c->dr + b * w);
    if (c->tolerance >= 0)
        sgm_oracle_lr_check(c->dl + b * w, c->dr + b * w, c->width, rows, c->tolerance, c->chk + b * w);
    else
        memcpy(c->chk + b * w, c->dl + b * w, (size_t)rows * w * sizeof(uint16_t));
}

static const int kDirs[8][2] = {
    {1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, 1}, {1, -1}, {-1, -1},
};

int sgm_oracle_run_threaded(const uint8_t* left, const uint8_t* right, int width, int height,
                            int win_w, int win_h, int ndisp, int npaths, int p1, int p2,
                            int lr_tolerance, int median3x3, int nthreads,
                            uint16_t* disp_left, uint16_t* disp_right, uint16_t* disp) {
    const size_t n = (size_t)width * height;
    const size_t nv = n * (size_t)ndisp;
    Ctx c;
    memset(&c, 0, sizeof(c));
    c.left = left;
    c.right = right;
    c.width = width;
    c.height = height;
    c.win_w = win_w;
    c.win_h = win_h;
    c.ndisp = ndisp;
    c.p1 = p1;
    c.p2 = p2;
    c.tolerance = lr_tolerance;
    c.cl = (uint64_t*)malloc(n * sizeof(uint64_t));
    c.cr = (uint64_t*)malloc(n * sizeof(uint64_t));
    c.cost = (uint8_t*)malloc(nv);
    c.path = (uint16_t*)malloc(nv * sizeof(uint16_t));
    c.sum = (uint32_t*)calloc(nv, sizeof(uint32_t));
    c.agg = (uint16_t*)malloc(nv * sizeof(uint16_t));
    c.starts = (int*)malloc(2 * (size_t)(width + height) * sizeof(int));
    c.dl = disp_left;
    c.dr = disp_right;
    c.chk = (uint16_t*)malloc(n * sizeof(uint16_t));
    int rc = 0;
    if (!c.cl || !c.cr || !c.cost || !c.path || !c.sum || !c.agg || !c.starts || !c.chk) {
        rc = -1;
        goto done;
    }
    parallel_for(nthreads, 2, census_part, &c);
    parallel_for(nthreads, height, cost_rows, &c);
    for (int r = 0; r < npaths; ++r) {
        c.dx = kDirs[r][0];
        c.dy = kDirs[r][1];
        long nstarts = 0;
        for (int y = 0; y < height; ++y)
            for (int x = 0; x < width; ++x)
                if (!inside(x - c.dx, y - c.dy, width, height)) {
                    c.starts[2 * nstarts] = x;
                    c.starts[2 * nstarts + 1] = y;
                    ++nstarts;
                }
        parallel_for(nthreads, nstarts, path_lines, &c);
        parallel_for(nthreads, (long)nv, add_path, &c);
    }
    parallel_for(nthreads, (long)nv, narrow_sum, &c);
    parallel_for(nthreads, height, select_rows, &c);
    if (median3x3)
        sgm_oracle_median3x3(c.chk, width, height, disp);
    else
        memcpy(disp, c.chk, n * sizeof(uint16_t));
done:
    free(c.chk);
    free(c.starts);
    free(c.agg);
    free(c.sum);
    free(c.path);
    free(c.cost);
    free(c.cr);
    free(c.cl);
    return rc;
}
