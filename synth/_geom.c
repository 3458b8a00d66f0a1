/*
 * Geometry helpers for the synthetic amorphous hydrocarbon boxes.
 *
 * This file produces INPUTS only (atom positions and neighbour pairs).  It
 * holds none of the solver's arithmetic and is shared by the CPU oracle and
 * the GPU path alike.
 *
 *   rsa_place      random sequential addition of n points in a periodic cube
 *                  of side L with a minimum pair distance dmin (minimum image),
 *                  drawing candidates from a splitmix64 stream (Steele, Lea,
 *                  Flood 2014) seeded by `seed`.
 *   count_pairs /
 *   fill_pairs     all unordered pairs I<J with minimum-image distance
 *                  r <= rcut, found with a linked cell list; pairs are emitted
 *                  sorted by (I, J).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t splitmix64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform double in [0,1) from the top 53 bits */
static inline double u01(uint64_t *s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

static inline double wrap_d(double d, double L) {
    /* minimum-image displacement component */
    d -= L * nearbyint(d / L);
    return d;
}

typedef struct {
    int nc;           /* cells per side */
    double cs;        /* cell side */
    int *head;        /* nc^3 */
    int *next;        /* n */
} cell_list;

static int cell_of(double x, double cs, int nc) {
    int c = (int)floor(x / cs);
    if (c < 0) c = 0;
    if (c >= nc) c = nc - 1;
    return c;
}

static int cl_init(cell_list *cl, double L, double rmin_cell, int n) {
    int nc = (int)floor(L / rmin_cell);
    if (nc < 1) nc = 1;
    if (nc > 1024) nc = 1024;
    cl->nc = nc;
    cl->cs = L / nc;
    size_t ncell = (size_t)nc * nc * nc;
    cl->head = (int *)malloc(ncell * sizeof(int));
    cl->next = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    if (!cl->head || !cl->next) return -1;
    for (size_t i = 0; i < ncell; ++i) cl->head[i] = -1;
    return 0;
}

static void cl_free(cell_list *cl) {
    free(cl->head);
    free(cl->next);
}

/* Returns 0 on success, -1 if max_tries candidates were not enough. */
int rsa_place(int n, double L, double dmin, uint64_t seed, int64_t max_tries, double *pos) {
    cell_list cl;
    if (cl_init(&cl, L, dmin, n) != 0) return -2;
    const int nc = cl.nc;
    const double d2 = dmin * dmin;
    uint64_t s = seed;
    int placed = 0;
    int64_t tries = 0;
    while (placed < n) {
        if (tries++ >= max_tries) { cl_free(&cl); return -1; }
        double x = u01(&s) * L, y = u01(&s) * L, z = u01(&s) * L;
        int cx = cell_of(x, cl.cs, nc), cy = cell_of(y, cl.cs, nc), cz = cell_of(z, cl.cs, nc);
        int ok = 1;
        int span = (nc >= 3) ? 1 : 0;
        for (int dx = -span; dx <= span && ok; ++dx)
            for (int dy = -span; dy <= span && ok; ++dy)
                for (int dz = -span; dz <= span && ok; ++dz) {
                    int ax = (cx + dx + nc) % nc, ay = (cy + dy + nc) % nc, az = (cz + dz + nc) % nc;
                    for (int a = cl.head[((size_t)ax * nc + ay) * nc + az]; a >= 0; a = cl.next[a]) {
                        double ddx = wrap_d(pos[3 * a] - x, L), ddy = wrap_d(pos[3 * a + 1] - y, L),
                               ddz = wrap_d(pos[3 * a + 2] - z, L);
                        if (ddx * ddx + ddy * ddy + ddz * ddz < d2) { ok = 0; break; }
                    }
                }
        if (nc < 3 && ok) {
            /* tiny boxes: brute force */
            for (int a = 0; a < placed && ok; ++a) {
                double ddx = wrap_d(pos[3 * a] - x, L), ddy = wrap_d(pos[3 * a + 1] - y, L),
                       ddz = wrap_d(pos[3 * a + 2] - z, L);
                if (ddx * ddx + ddy * ddy + ddz * ddz < d2) ok = 0;
            }
        }
        if (!ok) continue;
        pos[3 * placed] = x;
        pos[3 * placed + 1] = y;
        pos[3 * placed + 2] = z;
        size_t c = ((size_t)cx * nc + cy) * nc + cz;
        cl.next[placed] = cl.head[c];
        cl.head[c] = placed;
        ++placed;
    }
    cl_free(&cl);
    return 0;
}

/* Shared pair walker.  mode 0: count per atom I (pairs I<J) into cnt[I].
 * mode 1: fill, using row offsets off[I] (exclusive prefix of cnt) and writing
 * J into pj, r into pr and the minimum-image vector r_J - r_I into pd.
 * Pairs of one I are sorted by J afterwards by the caller's order guarantee:
 * we sort each row here with insertion sort (rows are short). */
static int walk_pairs(int n, const double *pos, double L, double rcut, int mode, int64_t *cnt,
                      const int64_t *off, int32_t *pj, double *pr, double *pd) {
    cell_list cl;
    if (cl_init(&cl, L, rcut, n) != 0) return -2;
    const int nc = cl.nc;
    for (int a = n - 1; a >= 0; --a) {
        int cx = cell_of(pos[3 * a], cl.cs, nc), cy = cell_of(pos[3 * a + 1], cl.cs, nc),
            cz = cell_of(pos[3 * a + 2], cl.cs, nc);
        size_t c = ((size_t)cx * nc + cy) * nc + cz;
        cl.next[a] = cl.head[c];
        cl.head[c] = a;
    }
    const double rc2 = rcut * rcut;
    int64_t *fillpos = NULL;
    if (mode == 1) {
        fillpos = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        if (!fillpos) { cl_free(&cl); return -2; }
        for (int i = 0; i < n; ++i) fillpos[i] = off[i];
    }
    for (int i = 0; i < n; ++i) {
        double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
        int cx = cell_of(x, cl.cs, nc), cy = cell_of(y, cl.cs, nc), cz = cell_of(z, cl.cs, nc);
        if (nc >= 3) {
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        int ax = (cx + dx + nc) % nc, ay = (cy + dy + nc) % nc, az = (cz + dz + nc) % nc;
                        for (int j = cl.head[((size_t)ax * nc + ay) * nc + az]; j >= 0; j = cl.next[j]) {
                            if (j <= i) continue;
                            double ddx = wrap_d(pos[3 * j] - x, L), ddy = wrap_d(pos[3 * j + 1] - y, L),
                                   ddz = wrap_d(pos[3 * j + 2] - z, L);
                            double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                            if (r2 > rc2) continue;
                            if (mode == 0) {
                                cnt[i]++;
                            } else {
                                int64_t p = fillpos[i]++;
                                pj[p] = j;
                                pr[p] = sqrt(r2);
                                pd[3 * p] = ddx;
                                pd[3 * p + 1] = ddy;
                                pd[3 * p + 2] = ddz;
                            }
                        }
                    }
        } else {
            for (int j = i + 1; j < n; ++j) {
                double ddx = wrap_d(pos[3 * j] - x, L), ddy = wrap_d(pos[3 * j + 1] - y, L),
                       ddz = wrap_d(pos[3 * j + 2] - z, L);
                double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                if (r2 > rc2) continue;
                if (mode == 0) {
                    cnt[i]++;
                } else {
                    int64_t p = fillpos[i]++;
                    pj[p] = j;
                    pr[p] = sqrt(r2);
                    pd[3 * p] = ddx;
                    pd[3 * p + 1] = ddy;
                    pd[3 * p + 2] = ddz;
                }
            }
        }
        if (mode == 1) {
            /* sort this row by j (insertion sort; rows hold ~20 entries) */
            int64_t b = off[i], e = fillpos[i];
            for (int64_t p = b + 1; p < e; ++p) {
                int32_t kj = pj[p];
                double kr = pr[p], k0 = pd[3 * p], k1 = pd[3 * p + 1], k2 = pd[3 * p + 2];
                int64_t q = p - 1;
                while (q >= b && pj[q] > kj) {
                    pj[q + 1] = pj[q];
                    pr[q + 1] = pr[q];
                    pd[3 * (q + 1)] = pd[3 * q];
                    pd[3 * (q + 1) + 1] = pd[3 * q + 1];
                    pd[3 * (q + 1) + 2] = pd[3 * q + 2];
                    --q;
                }
                pj[q + 1] = kj;
                pr[q + 1] = kr;
                pd[3 * (q + 1)] = k0;
                pd[3 * (q + 1) + 1] = k1;
                pd[3 * (q + 1) + 2] = k2;
            }
        }
    }
    free(fillpos);
    cl_free(&cl);
    return 0;
}

int count_pairs(int n, const double *pos, double L, double rcut, int64_t *cnt) {
    memset(cnt, 0, (size_t)n * sizeof(int64_t));
    return walk_pairs(n, pos, L, rcut, 0, cnt, NULL, NULL, NULL, NULL);
}

int fill_pairs(int n, const double *pos, double L, double rcut, const int64_t *off, int32_t *pj, double *pr,
               double *pd) {
    return walk_pairs(n, pos, L, rcut, 1, NULL, off, pj, pr, pd);
}
