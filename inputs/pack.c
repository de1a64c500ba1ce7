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
 */
#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double wrap(double x, double L)
{
    x -= L * floor(x / L);
    if (x >= L) x -= L;
    return x;
}

/* Returns the largest overlap after the last sweep; *iters gets the sweep count. */
double pack_relax(int n, const double *a, double *x, const double L[3], double tol, int maxiter,
                  double alpha, int *iters)
{
    double amax = 0.0;
    for (int i = 0; i < n; ++i) if (a[i] > amax) amax = a[i];
    int nc[3];
    for (int d = 0; d < 3; ++d) {
        nc[d] = (int)floor(L[d] / (2.0 * amax));
        if (nc[d] < 3) nc[d] = 1;
    }
    long ncell = (long)nc[0] * nc[1] * nc[2];
    int *cstart = (int *)malloc(sizeof(int) * (size_t)(ncell + 1));
    int *ccount = (int *)malloc(sizeof(int) * (size_t)ncell);
    int *cell = (int *)malloc(sizeof(int) * (size_t)n);
    int *sorted = (int *)malloc(sizeof(int) * (size_t)n);
    double *dx = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *ov = (double *)malloc(sizeof(double) * (size_t)n);
    double *xs = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *as = (double *)malloc(sizeof(double) * (size_t)n);
    double maxov = 0.0;
    int it;
    for (it = 0; it < maxiter; ++it) {
        memset(ccount, 0, sizeof(int) * (size_t)ncell);
        for (int i = 0; i < n; ++i) {
            int c[3];
            for (int d = 0; d < 3; ++d) {
                int q = (int)floor(x[3 * i + d] / L[d] * nc[d]);
                c[d] = q < 0 ? 0 : (q >= nc[d] ? nc[d] - 1 : q);
            }
            cell[i] = (c[2] * nc[1] + c[1]) * nc[0] + c[0];
            ccount[cell[i]]++;
        }
        cstart[0] = 0;
        for (long c = 0; c < ncell; ++c) cstart[c + 1] = cstart[c] + ccount[c];
        memset(ccount, 0, sizeof(int) * (size_t)ncell);
        for (int i = 0; i < n; ++i) sorted[cstart[cell[i]] + ccount[cell[i]]++] = i;

        /* cell-ordered copies, so that the candidate loop reads memory in order */
#pragma omp parallel for schedule(static)
        for (int q = 0; q < n; ++q) {
            const int i = sorted[q];
            for (int d = 0; d < 3; ++d) xs[3 * q + d] = x[3 * i + d];
            as[q] = a[i];
        }

#pragma omp parallel for schedule(static)
        for (int qi = 0; qi < n; ++qi) {
            int i = sorted[qi];
            int ci = cell[i];
            int cx = ci % nc[0], cy = (ci / nc[0]) % nc[1], cz = ci / (nc[0] * nc[1]);
            double acc[3] = {0, 0, 0};
            double mo = 0.0;
            for (int oz = (nc[2] == 1 ? 0 : -1); oz <= (nc[2] == 1 ? 0 : 1); ++oz)
                for (int oy = (nc[1] == 1 ? 0 : -1); oy <= (nc[1] == 1 ? 0 : 1); ++oy)
                    for (int ox = (nc[0] == 1 ? 0 : -1); ox <= (nc[0] == 1 ? 0 : 1); ++ox) {
                        int xx = (cx + ox + nc[0]) % nc[0];
                        int yy = (cy + oy + nc[1]) % nc[1];
                        int zz = (cz + oz + nc[2]) % nc[2];
                        int c = (zz * nc[1] + yy) * nc[0] + xx;
                        for (int q = cstart[c]; q < cstart[c + 1]; ++q) {
                            int j = sorted[q];
                            if (j == i) continue;
                            double r[3];
                            for (int d = 0; d < 3; ++d) {
                                double t = xs[3 * qi + d] - xs[3 * q + d];
                                r[d] = t - L[d] * rint(t / L[d]);
                            }
                            double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                            double sa = as[qi] + as[q];
                            if (d2 >= sa * sa) continue;
                            double dist = sqrt(d2);
                            double o = sa - dist;
                            if (o > mo) mo = o;
                            if (dist > 0.0) {
                                for (int d = 0; d < 3; ++d) acc[d] += 0.5 * o * r[d] / dist;
                            } else {
                                acc[0] += 0.5 * o * (i < j ? 1.0 : -1.0);
                            }
                        }
                    }
            for (int d = 0; d < 3; ++d) dx[3 * i + d] = alpha * acc[d];
            ov[i] = mo;
        }
        maxov = 0.0;
        for (int i = 0; i < n; ++i) if (ov[i] > maxov) maxov = ov[i];
        if (n >= 200000 && it % 100 == 0) {
            fprintf(stderr, "pack: n=%d sweep %d max overlap %.3e (tol %.1e)\n", n, it, maxov, tol);
            fflush(stderr);
        }
        if (maxov <= tol) break;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) x[3 * i + d] = wrap(x[3 * i + d] + dx[3 * i + d], L[d]);
    }
    if (iters) *iters = it;
    free(cstart); free(ccount); free(cell); free(sorted); free(dx); free(ov); free(xs); free(as);
    return maxov;
}
