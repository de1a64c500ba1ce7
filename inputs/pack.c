/*
 * pack.c -- seeded synthetic initial packings for the test and benchmark
 * workloads: spheres placed uniformly at random in a periodic box, then moved
 * apart by repeated overlap-removal sweeps until the largest overlap is below a
 * tolerance.  This is an input generator only; it holds none of the force law
 * or time stepping of the method and is shared, as data, by the CPU oracle and
 * the GPU library.
 *
 * Each sweep: for every sphere i, d_i = alpha * sum_j (overlap_ij / 2) n_ij
 * over the spheres j that overlap it (minimum image in an orthogonal periodic
 * box), then x_i += d_i for all i at once.  Jacobi sweeps make the result
 * independent of the thread count.
 *
 * The candidates j come from a neighbour list of the pairs closer than
 * a_i + a_j + skin, built from a cell list with the spheres in cell order and
 * rebuilt once the displacements since the build could have used up the skin
 * (twice the sum of the largest displacement of each sweep): every overlapping
 * pair is then in the list, so the sweeps are those of a full cell search.
 */
#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PACK_NB_CAP 64   /* list entries per sphere */

static double wrap(double x, double L)
{
    x -= L * floor(x / L);
    if (x >= L) x -= L;
    return x;
}

typedef struct {
    int n, nc[3];
    double L[3];
    int *cstart, *ccount, *cell, *perm, *orig, *tmp_i;
    double *tmp_x, *tmp_a;
} cells_t;

/* Wraps the positions xs (slot order) into the box, sorts the slots by cell (counting
 * sort, stable in slot order) and permutes xs, as and orig accordingly. */
static void sort_by_cell(cells_t *C, double *xs, double *as)
{
    const int n = C->n;
    const long ncell = (long)C->nc[0] * C->nc[1] * C->nc[2];
#pragma omp parallel for schedule(static)
    for (int q = 0; q < n; ++q) {
        int c[3];
        for (int d = 0; d < 3; ++d) {
            double v = wrap(xs[3 * q + d], C->L[d]);
            xs[3 * q + d] = v;
            int t = (int)floor(v / C->L[d] * C->nc[d]);
            c[d] = t < 0 ? 0 : (t >= C->nc[d] ? C->nc[d] - 1 : t);
        }
        C->cell[q] = (c[2] * C->nc[1] + c[1]) * C->nc[0] + c[0];
    }
    memset(C->ccount, 0, sizeof(int) * (size_t)ncell);
    for (int q = 0; q < n; ++q) C->ccount[C->cell[q]]++;
    C->cstart[0] = 0;
    for (long c = 0; c < ncell; ++c) C->cstart[c + 1] = C->cstart[c] + C->ccount[c];
    memset(C->ccount, 0, sizeof(int) * (size_t)ncell);
    for (int q = 0; q < n; ++q) C->perm[C->cstart[C->cell[q]] + C->ccount[C->cell[q]]++] = q;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        const int q = C->perm[k];
        for (int d = 0; d < 3; ++d) C->tmp_x[3 * k + d] = xs[3 * q + d];
        C->tmp_a[k] = as[q];
        C->tmp_i[k] = C->orig[q];
    }
    memcpy(xs, C->tmp_x, sizeof(double) * 3 * (size_t)n);
    memcpy(as, C->tmp_a, sizeof(double) * (size_t)n);
    memcpy(C->orig, C->tmp_i, sizeof(int) * (size_t)n);
}

/* Neighbour list (slots in cell order): for each slot k its partners j with
 * |x_k - x_j - shift| < a_k + a_j + skin, shift the periodic image offset.
 * Returns 0, or -1 when a sphere has more than PACK_NB_CAP partners. */
static int build_list(const cells_t *C, const double *xs, const double *as, double skin, int *nn, int *nb,
                      double *nsh)
{
    const int n = C->n;
    const int *nc = C->nc;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int k = 0; k < n; ++k) {
        int ci[3];
        for (int d = 0; d < 3; ++d) {
            int t = (int)floor(xs[3 * k + d] / C->L[d] * nc[d]);
            ci[d] = t < 0 ? 0 : (t >= nc[d] ? nc[d] - 1 : t);
        }
        int cnt = 0;
        for (int oz = (nc[2] == 1 ? 0 : -1); oz <= (nc[2] == 1 ? 0 : 1); ++oz)
            for (int oy = (nc[1] == 1 ? 0 : -1); oy <= (nc[1] == 1 ? 0 : 1); ++oy)
                for (int ox = (nc[0] == 1 ? 0 : -1); ox <= (nc[0] == 1 ? 0 : 1); ++ox) {
                    const int o[3] = {ox, oy, oz};
                    int cc[3];
                    for (int d = 0; d < 3; ++d) cc[d] = (ci[d] + o[d] + nc[d]) % nc[d];
                    const int c = (cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
                    for (int j = C->cstart[c]; j < C->cstart[c + 1]; ++j) {
                        if (j == k) continue;
                        double r[3], sh[3];
                        for (int d = 0; d < 3; ++d) {
                            const double t = xs[3 * k + d] - xs[3 * j + d];
                            sh[d] = -C->L[d] * rint(t / C->L[d]);   /* nearest image of j */
                            r[d] = t + sh[d];
                        }
                        const double rl = as[k] + as[j] + skin;
                        if (r[0] * r[0] + r[1] * r[1] + r[2] * r[2] >= rl * rl) continue;
                        if (cnt >= PACK_NB_CAP) { bad = 1; continue; }
                        nb[(size_t)k * PACK_NB_CAP + cnt] = j;
                        for (int d = 0; d < 3; ++d) nsh[((size_t)k * PACK_NB_CAP + cnt) * 3 + d] = -sh[d];
                        ++cnt;
                    }
                }
        nn[k] = cnt;
    }
    return bad ? -1 : 0;
}

/* Returns the largest overlap after the last sweep (-1 if a neighbour list
 * overflowed); *iters gets the sweep count. */
double pack_relax(int n, const double *a, double *x, const double L[3], double tol, int maxiter,
                  double alpha, int *iters)
{
    double amax = 0.0, amin = 1e300;
    for (int i = 0; i < n; ++i) {
        if (a[i] > amax) amax = a[i];
        if (a[i] < amin) amin = a[i];
    }
    const double skin = 0.25 * amin;
    cells_t C;
    C.n = n;
    for (int d = 0; d < 3; ++d) {
        C.L[d] = L[d];
        C.nc[d] = (int)floor(L[d] / (2.0 * amax + skin));
        if (C.nc[d] < 3) C.nc[d] = 1;
    }
    const long ncell = (long)C.nc[0] * C.nc[1] * C.nc[2];
    C.cstart = (int *)malloc(sizeof(int) * (size_t)(ncell + 1));
    C.ccount = (int *)malloc(sizeof(int) * (size_t)ncell);
    C.cell = (int *)malloc(sizeof(int) * (size_t)n);
    C.perm = (int *)malloc(sizeof(int) * (size_t)n);
    C.orig = (int *)malloc(sizeof(int) * (size_t)n);
    C.tmp_i = (int *)malloc(sizeof(int) * (size_t)n);
    C.tmp_x = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    C.tmp_a = (double *)malloc(sizeof(double) * (size_t)n);
    double *xs = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *as = (double *)malloc(sizeof(double) * (size_t)n);
    double *dx = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *ov = (double *)malloc(sizeof(double) * (size_t)n);
    double *mv = (double *)malloc(sizeof(double) * (size_t)n);
    int *nn = (int *)malloc(sizeof(int) * (size_t)n);
    int *nb = (int *)malloc(sizeof(int) * (size_t)n * PACK_NB_CAP);
    double *nsh = (double *)malloc(sizeof(double) * 3 * (size_t)n * PACK_NB_CAP);
    memcpy(xs, x, sizeof(double) * 3 * (size_t)n);
    memcpy(as, a, sizeof(double) * (size_t)n);
    for (int i = 0; i < n; ++i) C.orig[i] = i;

    double maxov = 0.0, moved = 2.0 * skin;   /* displacement bound since the last build */
    int it, lists = 0;
    for (it = 0; it < maxiter; ++it) {
        if (2.0 * moved >= skin) {
            sort_by_cell(&C, xs, as);
            if (build_list(&C, xs, as, skin, nn, nb, nsh) != 0) { maxov = -1.0; break; }
            moved = 0.0;
            ++lists;
        }
#pragma omp parallel for schedule(static)
        for (int k = 0; k < n; ++k) {
            double acc[3] = {0, 0, 0};
            double mo = 0.0;
            const double *xk = &xs[3 * k];
            for (int e = 0; e < nn[k]; ++e) {
                const size_t s = (size_t)k * PACK_NB_CAP + e;
                const int j = nb[s];
                double r[3];
                for (int d = 0; d < 3; ++d) r[d] = xk[d] - (xs[3 * j + d] + nsh[3 * s + d]);
                const double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                const double sa = as[k] + as[j];
                if (d2 >= sa * sa) continue;
                const double dist = sqrt(d2);
                const double olap = sa - dist;
                if (olap > mo) mo = olap;
                if (dist > 0.0) {
                    for (int d = 0; d < 3; ++d) acc[d] += 0.5 * olap * r[d] / dist;
                } else {
                    acc[0] += 0.5 * olap * (C.orig[k] < C.orig[j] ? 1.0 : -1.0);
                }
            }
            double m2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                dx[3 * k + d] = alpha * acc[d];
                m2 += dx[3 * k + d] * dx[3 * k + d];
            }
            ov[k] = mo;
            mv[k] = sqrt(m2);
        }
        maxov = 0.0;
        double mstep = 0.0;
        for (int k = 0; k < n; ++k) {
            if (ov[k] > maxov) maxov = ov[k];
            if (mv[k] > mstep) mstep = mv[k];
        }
        if (n >= 200000 && it % 100 == 0) {
            fprintf(stderr, "pack: n=%d sweep %d max overlap %.3e (tol %.1e), %d list builds\n", n, it, maxov, tol,
                    lists);
            fflush(stderr);
        }
        if (maxov <= tol) break;
#pragma omp parallel for schedule(static)
        for (int q = 0; q < 3 * n; ++q) xs[q] += dx[q];
        moved += mstep * (1.0 + 1e-12);
    }
    for (int k = 0; k < n; ++k)
        for (int d = 0; d < 3; ++d) x[3 * C.orig[k] + d] = wrap(xs[3 * k + d], L[d]);
    if (iters) *iters = it;
    free(C.cstart); free(C.ccount); free(C.cell); free(C.perm); free(C.orig); free(C.tmp_i); free(C.tmp_x);
    free(C.tmp_a); free(xs); free(as); free(dx); free(ov); free(mv); free(nn); free(nb); free(nsh);
    return maxov;
}
