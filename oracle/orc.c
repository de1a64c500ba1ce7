/*
 * orc.c -- plain, single-threaded FP64 reference ("oracle") of the pairwise
 * suspension model of Li, Royer & Ness, "Simulating the rheology of dense
 * suspensions using pairwise formulation of contact, lubrication and Brownian
 * forces" (arXiv 2307.13802).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * measured against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source with the HIP library.
 *
 * Build: gcc -std=c99 -O2 -ffp-contract=off -fPIC -shared (no fast-math), so
 * every +,-,*,/ and sqrt is one IEEE-754 correctly rounded FP64 operation.
 *
 * What it computes, per section of the paper:
 *   Sec. II, eq. (lang_force), (lang_torque): translational and rotational
 *       Langevin equations with particle inertia, I = (2/5) m a^2.
 *   Sec. II (footnote on the skin): velocity-Verlet time stepping.
 *   Sec. II.A, eq. (force_contact), (torque_contact): Hookean normal contact,
 *       tangential spring with history, Coulomb limit mu.
 *   Sec. II.A (last paragraph): contact stress -F (x) r / V.
 *   Sec. II.B, eq. (force_drag), (torque_drag): one-body Stokes drag.
 *   Sec. II.B, eq. (force_lub) with the X^A_11 and Y^A_11 scalars: squeeze
 *       and shear lubrication, regularised at xi_eff = 1e-3 and cut off for
 *       gaps xi > 0.05; lubrication stress -F (x) r / V.
 *   Sec. II.C, eq. (force_brownian_drag), (torque_brownian_drag),
 *       (force_brownian_lub): one-body and pairwise Brownian forces with
 *       amplitude sqrt(2 kT / dt) times the square root of the resistance.
 *   Sec. II.B (after eq. torque_drag): drag stresslet (20/3) pi eta a^3 E per
 *       particle, summed and divided by V.
 *   Sec. II.D: instantaneous Brownian stress -F^{B,L} (x) r / V.
 *   Sec. IV.D: total stress = hydrodynamic (lubrication + drag) + contact;
 *       Sec. II.E: relative viscosity eta_r = Sigma_xy / (eta gammadot).
 *   Sec. IV.F: short-ranged repulsion A/kappa exp(-h/kappa) n (switch rep_A).
 *   Sec. III.A, IV.B: pair-distance histograms and stress autocorrelations
 *       (the observables of g(r) and of the Green-Kubo integral).
 *   Sec. II.E: sheared periodic box; the tilted-box remap is represented by a
 *       Lees-Edwards offset (same image lattice, no effect on forces).
 *
 * Readings taken where the text is silent or garbled (each is also listed in
 * the design notes of the repository):
 *   r_ij = x_i - x_j (n points from j to i); this is the orientation under
 *       which the printed contact force is repulsive, the printed torque is
 *       lever-arm x force, and -F (x) r gives a positive viscosity.
 *   Velocity-dependent forces use the half-step velocities of velocity-Verlet.
 *   Tangential spring: Cundall-Strack (rotate into the current tangent plane
 *       keeping |s|, add the tangential contact-point velocity times dt, then
 *       truncate the stored spring at the Coulomb limit; strict '>').
 *   Pair Brownian forces act on exactly the lubrication pairs (xi <= xi_cut),
 *       overlapping pairs included (with xi_eff).
 *   Noise: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit seed,
 *       counter (step_lo, id_min, id_max, step_hi<<8 | stream); uniform
 *       u = (w + 0.5) 2^-32; Box-Muller pairs.  The force on the lower id is
 *       +F^{B,L}, on the higher id -F^{B,L}.
 *   U^inf = gammadot (y - Ly/2) e_x, Omega^inf = (0, 0, -gammadot/2).
 *   Stress is divided by the volume only.
 *   The repulsion (no cut-off in the paper) acts on pairs with gap up to 16
 *       kappa, where it has decayed to exp(-16) of its contact value.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* flags (test switches; the physical model has all terms on) */
#define ORC_FREEZE_X     0x1u  /* positions are not advanced               */
#define ORC_NO_LUB       0x2u  /* drop the lubrication force              */
#define ORC_NO_PAIR_BROWN 0x4u /* drop the pairwise Brownian force        */
#define ORC_NO_CONTACT   0x8u  /* drop the contact force                  */
#define ORC_NO_ONEBODY   0x10u /* drop one-body drag and Brownian terms   */
#define ORC_CELLS        0x20u /* find pairs with a cell list, not O(N^2) */
#define ORC_LUB_ROT      0x40u /* model switch: rotational lubrication couplings (Y^B, Y^C)
                                  and the pairwise Brownian torques of Sec. II.B-II.C */

typedef struct {
    double L[3];          /* box lengths Lx, Ly, Lz                         */
    double rho, eta, kn, kt, mu, kT, gammadot, dt;
    double xi_cut;        /* lubrication cut-off on the dimensionless gap   */
    double xi_min;        /* regularisation xi_eff                          */
    double rep_A;         /* short-ranged repulsion scale A (0 = none)      */
    uint64_t seed;        /* Philox key                                     */
    uint32_t flags;
    uint32_t pad;
} orc_params;

typedef struct {
    uint32_t i, j;        /* i < j (ids)                                    */
    double s[3];          /* tangential spring                              */
    int sliding;          /* 1 if the Coulomb limit was hit at the last update */
} orc_contact;

typedef struct {
    orc_params p;
    int n;
    double *a, *m, *I;            /* radius, mass, moment of inertia        */
    double *x, *v, *w;            /* 3n each, particle-major (x0,y0,z0,...) */
    double *F, *T;                /* last evaluated force / torque          */
    double *Fabs, *Tabs;          /* sum of pair-force norms + one-body norm */
    double s_le;                  /* Lees-Edwards offset                     */
    uint64_t k;                   /* step counter of the last evaluation     */
    orc_contact *c; int nc, capc; /* contact history, sorted by (i, j)       */
    uint32_t *pairs; int npairs, cappairs; /* interaction set of last eval   */
    double stress[27];            /* contact, lubrication, Brownian 3x3     */
    double drag[9];               /* drag stresslet (1/V) sum 20/3 pi eta a^3 E */
    double *disp;                 /* 3n: accumulated non-affine displacement */
} orc_state;

/* ------------------------------------------------------------------ */
/* Philox4x32-10, from the description in Salmon, Moraes, Dror & Shaw, */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11).              */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;   /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;   /* Weyl key bumps    */
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Three standard normals from one Philox block, Box-Muller (1958). */
void orc_gauss3(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, double g[3])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    const double two_m32 = 2.3283064365386963e-10; /* 2^-32 */
    double u0 = ((double)w[0] + 0.5) * two_m32;
    double u1 = ((double)w[1] + 0.5) * two_m32;
    double u2 = ((double)w[2] + 0.5) * two_m32;
    double u3 = ((double)w[3] + 0.5) * two_m32;
    double r0 = sqrt(-2.0 * log(u0));
    double r1 = sqrt(-2.0 * log(u2));
    g[0] = r0 * cos((2.0 * ORC_PI) * u1);
    g[1] = r0 * sin((2.0 * ORC_PI) * u1);
    g[2] = r1 * cos((2.0 * ORC_PI) * u3);
}

/* Noise streams in the last counter word. */
#define ORC_STREAM_PAIR_FORCE 0u
#define ORC_STREAM_PAIR_TORQUE 1u
#define ORC_STREAM_ONE_FORCE  2u
#define ORC_STREAM_ONE_TORQUE 3u

static void gauss_pair(const orc_params *p, uint64_t k, uint32_t i, uint32_t j, double g[3])
{
    orc_gauss3(p->seed, (uint32_t)k, i, j, ((uint32_t)(k >> 32) << 8) | ORC_STREAM_PAIR_FORCE, g);
}

static void gauss_pair_torque(const orc_params *p, uint64_t k, uint32_t i, uint32_t j, double g[3])
{
    orc_gauss3(p->seed, (uint32_t)k, i, j, ((uint32_t)(k >> 32) << 8) | ORC_STREAM_PAIR_TORQUE, g);
}

static void gauss_one(const orc_params *p, uint64_t k, uint32_t i, uint32_t stream, double g[3])
{
    orc_gauss3(p->seed, (uint32_t)k, i, 0xFFFFFFFFu, ((uint32_t)(k >> 32) << 8) | stream, g);
}

/* ------------------------------------------------------------------ */
/* Lubrication scalars, Sec. II.B: X^A_11 and Y^A_11 exactly as printed,  */
/* with beta = a_j / a_i, prefactor 6 pi eta a_i, and xi the regularised */
/* dimensionless gap.                                                   */
/* ------------------------------------------------------------------ */
void orc_lub_scalars(double eta, double ai, double aj, double xi, double *XA, double *YA)
{
    double beta = aj / ai;
    double opb = 1.0 + beta;
    double opb3 = opb * opb * opb;
    double lg = log(1.0 / xi);
    double pre = 6.0 * ORC_PI * eta * ai;
    *XA = pre * ((2.0 * beta * beta) / opb3 * (1.0 / xi)
                 + (beta * (1.0 + 7.0 * beta + beta * beta)) / (5.0 * opb3) * lg);
    *YA = pre * ((4.0 * beta * (2.0 + beta + 2.0 * beta * beta)) / (15.0 * opb3) * lg);
}

/* Rotational lubrication scalars, Sec. II.B, exactly as printed: Y^B_11,
 * Y^B_21 (prefactors -4 pi eta a_i^2, -4 pi eta a_j^2) and Y^C_11, Y^C_12,
 * Y^C_21, Y^C_22 (prefactors 8 pi eta a_i^3, 8 pi eta a_j^3), beta = a_j/a_i. */
void orc_lub_rot_scalars(double eta, double ai, double aj, double xi, double out[6])
{
    double beta = aj / ai, ib = ai / aj;
    double lg = log(1.0 / xi);
    out[0] = -4.0 * ORC_PI * eta * ai * ai * (beta * (4.0 + beta) / (5.0 * (1.0 + beta) * (1.0 + beta))) * lg;
    out[1] = -4.0 * ORC_PI * eta * aj * aj * (ib * (4.0 + ib) / (5.0 * (1.0 + ib) * (1.0 + ib))) * lg;
    out[2] = 8.0 * ORC_PI * eta * ai * ai * ai * (2.0 * beta / (5.0 * (1.0 + beta))) * lg;
    out[3] = 8.0 * ORC_PI * eta * ai * ai * ai * (beta * beta / (10.0 * (1.0 + beta))) * lg;
    out[4] = 8.0 * ORC_PI * eta * aj * aj * aj * (ib * ib / (10.0 * (1.0 + ib))) * lg;
    out[5] = 8.0 * ORC_PI * eta * aj * aj * aj * (2.0 * ib / (5.0 * (1.0 + ib))) * lg;
}

/* ------------------------------------------------------------------ */
/* Sheared periodic box, Sec. II.E, as a Lees-Edwards offset s.          */
/* ------------------------------------------------------------------ */
static double nearest(double t) { return rint(t); }

/* Minimum image of x_i - x_j.  Returns k_y, the number of Ly periods
 * crossed; the image of j is displaced by k_y (s, Ly, 0). */
static int min_image(const orc_params *p, double s_le, const double *xi, const double *xj, double d[3])
{
    const double Lx = p->L[0], Ly = p->L[1], Lz = p->L[2];
    double dy = xi[1] - xj[1];
    int ky = (int)nearest(dy / Ly);
    dy = dy - (double)ky * Ly;
    double dx = (xi[0] - xj[0]) - (double)ky * s_le;
    dx = dx - Lx * nearest(dx / Lx);
    double dz = xi[2] - xj[2];
    dz = dz - Lz * nearest(dz / Lz);
    d[0] = dx; d[1] = dy; d[2] = dz;
    return ky;
}

static double dot3(const double a[3], const double b[3]) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------------ */
/* contact history: sorted array keyed by (i, j), i < j                  */
/* ------------------------------------------------------------------ */
static int contact_find(const orc_contact *c, int nc, uint32_t i, uint32_t j)
{
    int lo = 0, hi = nc - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (c[mid].i == i && c[mid].j == j) return mid;
        if (c[mid].i < i || (c[mid].i == i && c[mid].j < j)) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static int contact_cmp(const void *pa, const void *pb)
{
    const orc_contact *a = (const orc_contact *)pa, *b = (const orc_contact *)pb;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    return 0;
}

static int pair_cmp(const void *pa, const void *pb)
{
    const uint32_t *a = (const uint32_t *)pa, *b = (const uint32_t *)pb;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* One unordered pair, i < j.  Sec. II.A-II.D.                           */
/* ------------------------------------------------------------------ */
typedef struct {
    orc_contact *cnew; int ncnew, capcnew;
    const orc_contact *cold; int ncold;
    int overflow;
} contact_io;

/* Range of the short-ranged repulsion of Sec. IV.F: it acts on every pair with
 * gap h <= ORC_REP_RANGE * kappa, kappa = 0.01 (a_i + a_j), where it has decayed
 * to exp(-16) ~ 1e-7 of its contact value (the paper states no cut-off), i.e.
 * |r| <= (a_i + a_j) (1 + ORC_REP_RANGE * 0.01). */
#define ORC_REP_RANGE 16.0

static void repulsion_force(const orc_params *p, double sa, double dist, const double n[3], double FC[3])
{
    /* Sec. IV.F: A/kappa exp((a_i + a_j - |r|)/kappa) n, kappa = 0.01 (a_i + a_j); an
       interparticle force, kept with the contact force (and the contact stress) */
    double kappa = 0.01 * sa;
    double fr = p->rep_A / kappa * exp((sa - dist) / kappa);
    for (int d = 0; d < 3; ++d) FC[d] += fr * n[d];
}

static void pair_force(orc_state *S, int i, int j, contact_io *io)
{
    const orc_params *p = &S->p;
    double r[3];
    int ky = min_image(p, S->s_le, &S->x[3 * i], &S->x[3 * j], r);
    double d2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    double sa = S->a[i] + S->a[j];
    double rc = sa * (1.0 + 0.5 * p->xi_cut);
    if (!(d2 <= rc * rc)) {
        /* gap xi > xi_cut: no lubrication pair; only the repulsion may act */
        double rr = sa * (1.0 + ORC_REP_RANGE * 0.01);
        if (!(p->rep_A > 0.0) || !(d2 <= rr * rr)) return;
        double dist = sqrt(d2);
        double n[3] = {r[0] / dist, r[1] / dist, r[2] / dist};
        double FC[3] = {0, 0, 0};
        repulsion_force(p, sa, dist, n, FC);
        double V = p->L[0] * p->L[1] * p->L[2];
        for (int d = 0; d < 3; ++d) {
            S->F[3 * i + d] += FC[d];
            S->F[3 * j + d] -= FC[d];
        }
        double fn = sqrt(dot3(FC, FC));
        S->Fabs[i] += fn;
        S->Fabs[j] += fn;
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be) S->stress[0 + 3 * al + be] -= FC[al] * r[be] / V;
        return;
    }

    if (S->npairs >= S->cappairs) {
        S->cappairs = S->cappairs ? 2 * S->cappairs : 1024;
        S->pairs = (uint32_t *)realloc(S->pairs, (size_t)S->cappairs * 2 * sizeof(uint32_t));
    }
    S->pairs[2 * S->npairs] = (uint32_t)i; S->pairs[2 * S->npairs + 1] = (uint32_t)j; S->npairs++;

    double dist = sqrt(d2);
    double n[3] = {r[0] / dist, r[1] / dist, r[2] / dist};
    double h = dist - sa;
    double xi = (2.0 * h) / sa;
    double xie = xi < p->xi_min ? p->xi_min : xi;
    double XA, YA;
    orc_lub_scalars(p->eta, S->a[i], S->a[j], xie, &XA, &YA);

    /* velocity of j's image: Lees-Edwards jump of k_y gammadot Ly along x */
    double Uj[3] = {S->v[3 * j] + (double)ky * (p->gammadot * p->L[1]), S->v[3 * j + 1], S->v[3 * j + 2]};
    const double *vi = &S->v[3 * i];
    double FL[3] = {0, 0, 0}, FB[3] = {0, 0, 0}, FC[3] = {0, 0, 0};

    if (!(p->flags & ORC_NO_LUB)) {
        /* eq. (force_lub): (X^A N + Y^A T)(U_j - U_i) */
        double ur[3] = {Uj[0] - vi[0], Uj[1] - vi[1], Uj[2] - vi[2]};
        double un = dot3(n, ur);
        for (int d = 0; d < 3; ++d) FL[d] = XA * (un * n[d]) + YA * (ur[d] - un * n[d]);
    }
    double th[3] = {0, 0, 0};
    if (!(p->flags & ORC_NO_PAIR_BROWN)) {
        /* eq. (force_brownian_lub): sqrt(2kT/dt) (sqrt(X^A) N + sqrt(Y^A) T) theta */
        gauss_pair(p, S->k, (uint32_t)i, (uint32_t)j, th);
        double b = sqrt(2.0 * p->kT / p->dt);
        double tn = dot3(n, th);
        double sx = sqrt(XA), sy = sqrt(YA);
        for (int d = 0; d < 3; ++d) FB[d] = b * (sx * (tn * n[d]) + sy * (th[d] - tn * n[d]));
    }
    if (p->flags & ORC_LUB_ROT) {
        /* The rotational couplings are printed for n_ij pointing from i to j (the text's
           convention); with n from j to i (the reading under which the printed contact force
           repels) that vector is -n.  Both the lubrication and the Brownian parts act on the
           lubrication pairs. */
        double Y[6];
        orc_lub_rot_scalars(p->eta, S->a[i], S->a[j], xie, Y);
        const double YB11 = Y[0], YB21 = Y[1], YC11 = Y[2], YC12 = Y[3], YC21 = Y[4], YC22 = Y[5];
        double nij[3] = {-n[0], -n[1], -n[2]};
        const double *wi = &S->w[3 * i], *wj = &S->w[3 * j];
        double Ti[3] = {0, 0, 0}, Tj[3] = {0, 0, 0};
        if (!(p->flags & ORC_NO_LUB)) {
            /* eq. (force_lub), rotational part: Y^B_11 (Omega_i x n_ij) + Y^B_21 (Omega_j x n_ij) */
            double ci[3], cj[3];
            cross3(wi, nij, ci);
            cross3(wj, nij, cj);
            for (int d = 0; d < 3; ++d) FL[d] += YB11 * ci[d] + YB21 * cj[d];
            /* eq. (torque_lub1), (torque_lub2) */
            double ur[3] = {Uj[0] - vi[0], Uj[1] - vi[1], Uj[2] - vi[2]};
            double urn[3];
            cross3(ur, nij, urn);
            double oi[3], oj[3];
            for (int d = 0; d < 3; ++d) {
                oi[d] = YC11 * wi[d] + YC12 * wj[d];
                oj[d] = YC21 * wi[d] + YC22 * wj[d];
            }
            double oin = dot3(n, oi), ojn = dot3(n, oj);
            for (int d = 0; d < 3; ++d) {
                Ti[d] += YB11 * urn[d] - (oi[d] - oin * n[d]);
                Tj[d] += YB21 * urn[d] - (oj[d] - ojn * n[d]);
            }
        }
        if (!(p->flags & ORC_NO_PAIR_BROWN)) {
            /* eq. (torque_brownian_lub1), (torque_brownian_lub2): the force's theta and a
               second vector chi (stream 1); a negative radicand is read as zero */
            double chi[3];
            gauss_pair_torque(p, S->k, (uint32_t)i, (uint32_t)j, chi);
            double b = sqrt(2.0 * p->kT / p->dt);
            double thn[3];
            cross3(th, nij, thn);
            double cn = dot3(n, chi);
            double ri = YC11 - YB11 * YB11 / YA, rj = YC22 - YB21 * YB21 / YA;
            double si = ri > 0.0 ? sqrt(ri) : 0.0, sj = rj > 0.0 ? sqrt(rj) : 0.0;
            double sya = sqrt(YA);
            for (int d = 0; d < 3; ++d) {
                double tchi = chi[d] - cn * n[d];
                Ti[d] += b * (YB11 / sya * thn[d] + si * tchi);
                Tj[d] += b * (YB21 / sya * thn[d] + sj * tchi);
            }
        }
        for (int d = 0; d < 3; ++d) {
            S->T[3 * i + d] += Ti[d];
            S->T[3 * j + d] += Tj[d];
        }
        S->Tabs[i] += norm3(Ti);
        S->Tabs[j] += norm3(Tj);
    }
    if (h < 0.0 && !(p->flags & ORC_NO_CONTACT)) {
        /* eq. (force_contact), (torque_contact) with the Coulomb limit */
        double delta = -h;
        double s[3] = {0, 0, 0};
        int idx = contact_find(io->cold, io->ncold, (uint32_t)i, (uint32_t)j);
        if (idx >= 0) { s[0] = io->cold[idx].s[0]; s[1] = io->cold[idx].s[1]; s[2] = io->cold[idx].s[2]; }
        /* relative velocity of the contact point of i with respect to j */
        const double *wi = &S->w[3 * i], *wj = &S->w[3 * j];
        double aw[3];
        for (int d = 0; d < 3; ++d) aw[d] = S->a[i] * wi[d] + S->a[j] * wj[d];
        double awn[3];
        cross3(aw, n, awn);
        double vc[3];
        for (int d = 0; d < 3; ++d) vc[d] = (vi[d] - Uj[d]) - awn[d];
        double vcn = dot3(n, vc);
        double vt[3];
        for (int d = 0; d < 3; ++d) vt[d] = vc[d] - vcn * n[d];
        /* keep the spring in the current tangent plane, preserving its length */
        double sn = dot3(n, s);
        double pr[3];
        for (int d = 0; d < 3; ++d) pr[d] = s[d] - sn * n[d];
        double ps = norm3(pr);
        if (ps > 0.0) {
            double ss = norm3(s);
            double fac = ss / ps;
            for (int d = 0; d < 3; ++d) s[d] = pr[d] * fac;
        } else {
            for (int d = 0; d < 3; ++d) s[d] = pr[d];
        }
        for (int d = 0; d < 3; ++d) s[d] = s[d] + p->dt * vt[d];
        /* Coulomb: |k_t s| <= mu k_n delta; beyond it the spring is truncated */
        double ftmax = p->mu * p->kn * delta;
        double sl = norm3(s);
        int sliding = 0;
        if (p->kt * sl > ftmax) {
            double fac = ftmax / (p->kt * sl);
            for (int d = 0; d < 3; ++d) s[d] = s[d] * fac;
            sliding = 1;
        }
        double ks[3] = {p->kt * s[0], p->kt * s[1], p->kt * s[2]};
        for (int d = 0; d < 3; ++d) FC[d] = (p->kn * delta) * n[d] - ks[d];
        double nks[3];
        cross3(n, ks, nks);
        for (int d = 0; d < 3; ++d) {
            S->T[3 * i + d] += S->a[i] * nks[d];
            S->T[3 * j + d] += S->a[j] * nks[d];
        }
        if (io->ncnew >= io->capcnew) {
            io->capcnew = io->capcnew ? 2 * io->capcnew : 1024;
            io->cnew = (orc_contact *)realloc(io->cnew, (size_t)io->capcnew * sizeof(orc_contact));
        }
        orc_contact *cn = &io->cnew[io->ncnew++];
        cn->i = (uint32_t)i; cn->j = (uint32_t)j;
        cn->s[0] = s[0]; cn->s[1] = s[1]; cn->s[2] = s[2];
        cn->sliding = sliding;
        double tnorm = norm3(nks);
        S->Tabs[i] += S->a[i] * tnorm;
        S->Tabs[j] += S->a[j] * tnorm;
    }

    if (p->rep_A > 0.0) repulsion_force(p, sa, dist, n, FC);
    double V = p->L[0] * p->L[1] * p->L[2];
    for (int d = 0; d < 3; ++d) {
        double f = FL[d] + FB[d] + FC[d];
        S->F[3 * i + d] += f;
        S->F[3 * j + d] -= f;
    }
    double fn = sqrt(dot3(FL, FL)) + sqrt(dot3(FB, FB)) + sqrt(dot3(FC, FC));
    S->Fabs[i] += fn;
    S->Fabs[j] += fn;
    /* Sec. II.A, II.B, II.D: Sigma^X_ab -= F^X_a r_b / V for the pair once */
    for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be) {
            S->stress[0 + 3 * al + be] -= FC[al] * r[be] / V;
            S->stress[9 + 3 * al + be] -= FL[al] * r[be] / V;
            S->stress[18 + 3 * al + be] -= FB[al] * r[be] / V;
        }
}

/* ------------------------------------------------------------------ */
/* Forces(state, k): all pairs, then the one-body terms.                  */
/* ------------------------------------------------------------------ */
static int cells_dim(double L, double w) { int n = (int)floor(L / w); return n < 3 ? 1 : n; }

static void all_pairs(orc_state *S, contact_io *io)
{
    const int n = S->n;
    if (!(S->p.flags & ORC_CELLS)) {
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) pair_force(S, i, j, io);
        return;
    }
    /* simple cell list: cells no smaller than the largest interaction range;
     * rows that wrap across the sheared y boundary scan every x cell, so no
     * shift bookkeeping is needed; pairs are taken once with i < j. */
    double amax = 0.0;
    for (int i = 0; i < n; ++i) if (S->a[i] > amax) amax = S->a[i];
    double c = 1.0 + 0.5 * S->p.xi_cut;
    if (S->p.rep_A > 0.0 && 1.0 + ORC_REP_RANGE * 0.01 > c) c = 1.0 + ORC_REP_RANGE * 0.01;
    double rmax = 2.0 * amax * c;
    int nc[3];
    for (int d = 0; d < 3; ++d) nc[d] = cells_dim(S->p.L[d], rmax);
    int ncell = nc[0] * nc[1] * nc[2];
    int *head = (int *)malloc(sizeof(int) * (size_t)ncell);
    int *next = (int *)malloc(sizeof(int) * (size_t)n);
    int *cidx = (int *)malloc(sizeof(int) * 3 * (size_t)n);
    for (int c = 0; c < ncell; ++c) head[c] = -1;
    for (int i = n - 1; i >= 0; --i) {
        int ci[3];
        for (int d = 0; d < 3; ++d) {
            int q = (int)floor(S->x[3 * i + d] / S->p.L[d] * nc[d]);
            if (q < 0) q = 0;
            if (q >= nc[d]) q = nc[d] - 1;
            ci[d] = q; cidx[3 * i + d] = q;
        }
        int c = (ci[2] * nc[1] + ci[1]) * nc[0] + ci[0];
        next[i] = head[c]; head[c] = i;
    }
    for (int i = 0; i < n; ++i) {
        int cx = cidx[3 * i], cy = cidx[3 * i + 1], cz = cidx[3 * i + 2];
        int oy_lo = nc[1] == 1 ? 0 : -1, oy_hi = nc[1] == 1 ? 0 : 1;
        int oz_lo = nc[2] == 1 ? 0 : -1, oz_hi = nc[2] == 1 ? 0 : 1;
        for (int oz = oz_lo; oz <= oz_hi; ++oz)
            for (int oy = oy_lo; oy <= oy_hi; ++oy) {
                int yy = cy + oy;
                int wraps = (yy < 0 || yy >= nc[1]);
                yy = (yy + nc[1]) % nc[1];
                int zz = (cz + oz + nc[2]) % nc[2];
                int xlo, xhi;
                if (wraps || nc[0] == 1) { xlo = 0; xhi = nc[0] - 1; }
                else { xlo = cx - 1; xhi = cx + 1; }
                for (int ox = xlo; ox <= xhi; ++ox) {
                    int xx = (wraps || nc[0] == 1) ? ox : (ox + nc[0]) % nc[0];
                    int c = (zz * nc[1] + yy) * nc[0] + xx;
                    for (int j = head[c]; j >= 0; j = next[j])
                        if (j > i) pair_force(S, i, j, io);
                }
            }
    }
    free(head); free(next); free(cidx);
}

static void forces(orc_state *S)
{
    const orc_params *p = &S->p;
    const int n = S->n;
    memset(S->F, 0, sizeof(double) * 3 * (size_t)n);
    memset(S->T, 0, sizeof(double) * 3 * (size_t)n);
    memset(S->Fabs, 0, sizeof(double) * (size_t)n);
    memset(S->Tabs, 0, sizeof(double) * (size_t)n);
    memset(S->stress, 0, sizeof(S->stress));
    memset(S->drag, 0, sizeof(S->drag));
    S->npairs = 0;

    contact_io io = {NULL, 0, 0, S->c, S->nc, 0};
    all_pairs(S, &io);
    qsort(io.cnew, (size_t)io.ncnew, sizeof(orc_contact), contact_cmp);
    qsort(S->pairs, (size_t)S->npairs, 2 * sizeof(uint32_t), pair_cmp);
    free(S->c);
    S->c = io.cnew; S->nc = io.ncnew; S->capc = io.capcnew;

    if (!(p->flags & ORC_NO_ONEBODY)) {
        /* eq. (force_drag), (torque_drag), (force_brownian_drag), (torque_brownian_drag) */
        double b = sqrt(2.0 * p->kT / p->dt);
        for (int i = 0; i < n; ++i) {
            double zeta = 6.0 * ORC_PI * p->eta * S->a[i];
            double zr = 8.0 * ORC_PI * p->eta * S->a[i] * S->a[i] * S->a[i];
            double Uinf[3] = {p->gammadot * (S->x[3 * i + 1] - 0.5 * p->L[1]), 0.0, 0.0};
            double Oinf[3] = {0.0, 0.0, -0.5 * p->gammadot};
            double psi[3], phi[3];
            gauss_one(p, S->k, (uint32_t)i, ORC_STREAM_ONE_FORCE, psi);
            gauss_one(p, S->k, (uint32_t)i, ORC_STREAM_ONE_TORQUE, phi);
            double sz = sqrt(zeta), szr = sqrt(zr);
            double fd[3], td[3];
            for (int d = 0; d < 3; ++d) {
                double f = zeta * (Uinf[d] - S->v[3 * i + d]) + b * sz * psi[d];
                double t = zr * (Oinf[d] - S->w[3 * i + d]) + b * szr * phi[d];
                S->F[3 * i + d] += f;
                S->T[3 * i + d] += t;
                fd[d] = f; td[d] = t;
            }
            S->Fabs[i] += norm3(fd);
            S->Tabs[i] += norm3(td);
        }
        /* Sec. II.B: the drag force gives particle i the stress (20/3) pi eta a_i^3 E, with
           E the symmetric part of grad U^inf (only dU_x/dy = gammadot is nonzero) */
        double G[9] = {0, p->gammadot, 0, 0, 0, 0, 0, 0, 0};   /* G[3a+b] = dU_a/dx_b */
        double V = p->L[0] * p->L[1] * p->L[2];
        for (int i = 0; i < n; ++i) {
            double c = (20.0 / 3.0) * ORC_PI * p->eta * S->a[i] * S->a[i] * S->a[i];
            for (int al = 0; al < 3; ++al)
                for (int be = 0; be < 3; ++be) S->drag[3 * al + be] += c * 0.5 * (G[3 * al + be] + G[3 * be + al]);
        }
        for (int k = 0; k < 9; ++k) S->drag[k] /= V;
    }
}

/* ------------------------------------------------------------------ */
/* Time step n -> n+1 (velocity-Verlet, Sec. II).                        */
/* ------------------------------------------------------------------ */
static void kick(orc_state *S)
{
    const double dt = S->p.dt;
    for (int i = 0; i < S->n; ++i)
        for (int d = 0; d < 3; ++d) {
            S->v[3 * i + d] += (0.5 * dt / S->m[i]) * S->F[3 * i + d];
            S->w[3 * i + d] += (0.5 * dt / S->I[i]) * S->T[3 * i + d];
        }
}

static void step(orc_state *S)
{
    const orc_params *p = &S->p;
    const double Lx = p->L[0], Ly = p->L[1], Lz = p->L[2];
    kick(S);
    if (!(p->flags & ORC_FREEZE_X)) {
        /* non-affine displacement of the drift: dt v minus the imposed flow integrated along
           the straight path, gammadot (y(t) - Ly/2) e_x with y(t) = y + v_y t */
        for (int i = 0; i < S->n; ++i) {
            const double *x = &S->x[3 * i], *v = &S->v[3 * i];
            double ux = p->gammadot * (x[1] - 0.5 * Ly) + 0.5 * p->gammadot * p->dt * v[1];
            S->disp[3 * i] += p->dt * (v[0] - ux);
            S->disp[3 * i + 1] += p->dt * v[1];
            S->disp[3 * i + 2] += p->dt * v[2];
        }
        for (int q = 0; q < 3 * S->n; ++q) S->x[q] += p->dt * S->v[q];
    }
    S->s_le = S->s_le + p->gammadot * Ly * p->dt;
    S->s_le = S->s_le - Lx * floor(S->s_le / Lx);
    if (!(p->flags & ORC_FREEZE_X)) {
        for (int i = 0; i < S->n; ++i) {
            double *x = &S->x[3 * i];
            if (x[1] >= Ly) { x[1] -= Ly; x[0] -= S->s_le; S->v[3 * i] -= p->gammadot * Ly; }
            else if (x[1] < 0.0) {
                x[1] += Ly; x[0] += S->s_le; S->v[3 * i] += p->gammadot * Ly;
                if (x[1] >= Ly) x[1] = 0.0;   /* -tiny + Ly rounded up to Ly */
            }
            x[0] -= Lx * floor(x[0] / Lx);
            x[2] -= Lz * floor(x[2] / Lz);
            /* floor-based wrapping can land exactly on L after rounding */
            if (x[0] >= Lx) x[0] -= Lx;
            if (x[2] >= Lz) x[2] -= Lz;
        }
    }
    S->k += 1;
    forces(S);
    kick(S);
}

/* ------------------------------------------------------------------ */
/* C ABI for the Python test harness                                     */
/* ------------------------------------------------------------------ */
orc_state *orc_new(const orc_params *p, int n, const double *a, const double *x, const double *v,
                   const double *w, double s_le, uint64_t k, int nc, const uint32_t *c_ij,
                   const double *c_s, const double *F, const double *T)
{
    orc_state *S = (orc_state *)calloc(1, sizeof(orc_state));
    S->p = *p; S->n = n;
    S->a = (double *)malloc(sizeof(double) * (size_t)n);
    S->m = (double *)malloc(sizeof(double) * (size_t)n);
    S->I = (double *)malloc(sizeof(double) * (size_t)n);
    S->x = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    S->v = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    S->w = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    S->F = (double *)calloc(3 * (size_t)n, sizeof(double));
    S->T = (double *)calloc(3 * (size_t)n, sizeof(double));
    S->Fabs = (double *)calloc((size_t)n, sizeof(double));
    S->Tabs = (double *)calloc((size_t)n, sizeof(double));
    S->disp = (double *)calloc(3 * (size_t)n, sizeof(double));
    for (int i = 0; i < n; ++i) {
        S->a[i] = a[i];
        S->m[i] = (4.0 / 3.0) * ORC_PI * p->rho * a[i] * a[i] * a[i];   /* Sec. II */
        S->I[i] = 0.4 * S->m[i] * a[i] * a[i];                          /* (2/5) m a^2 */
    }
    memcpy(S->x, x, sizeof(double) * 3 * (size_t)n);
    memcpy(S->v, v, sizeof(double) * 3 * (size_t)n);
    memcpy(S->w, w, sizeof(double) * 3 * (size_t)n);
    S->s_le = s_le; S->k = k;
    S->nc = nc; S->capc = nc;
    S->c = nc ? (orc_contact *)malloc(sizeof(orc_contact) * (size_t)nc) : NULL;
    for (int q = 0; q < nc; ++q) {
        S->c[q].i = c_ij[2 * q]; S->c[q].j = c_ij[2 * q + 1];
        S->c[q].s[0] = c_s[3 * q]; S->c[q].s[1] = c_s[3 * q + 1]; S->c[q].s[2] = c_s[3 * q + 2];
        S->c[q].sliding = 0;
    }
    if (nc) qsort(S->c, (size_t)nc, sizeof(orc_contact), contact_cmp);
    if (F && T) {
        memcpy(S->F, F, sizeof(double) * 3 * (size_t)n);
        memcpy(S->T, T, sizeof(double) * 3 * (size_t)n);
    } else {
        forces(S);   /* forces at creation, with the given velocities */
    }
    return S;
}

void orc_free(orc_state *S)
{
    if (!S) return;
    free(S->a); free(S->m); free(S->I); free(S->x); free(S->v); free(S->w);
    free(S->F); free(S->T); free(S->Fabs); free(S->Tabs); free(S->c); free(S->pairs); free(S->disp);
    free(S);
}

/* Runs nsteps; if series is not NULL it receives 27 doubles per step. */
void orc_step(orc_state *S, long nsteps, double *series)
{
    for (long t = 0; t < nsteps; ++t) {
        step(S);
        if (series) memcpy(series + 27 * t, S->stress, sizeof(S->stress));
    }
}

/* Re-evaluates forces on the current state at the current step counter. */
void orc_eval(orc_state *S) { forces(S); }

void orc_get_state(const orc_state *S, double *x, double *v, double *w, double *F, double *T,
                   double *s_le, uint64_t *k)
{
    size_t b = sizeof(double) * 3 * (size_t)S->n;
    if (x) memcpy(x, S->x, b);
    if (v) memcpy(v, S->v, b);
    if (w) memcpy(w, S->w, b);
    if (F) memcpy(F, S->F, b);
    if (T) memcpy(T, S->T, b);
    if (s_le) *s_le = S->s_le;
    if (k) *k = S->k;
}

void orc_get_norms(const orc_state *S, double *Fabs, double *Tabs)
{
    memcpy(Fabs, S->Fabs, sizeof(double) * (size_t)S->n);
    memcpy(Tabs, S->Tabs, sizeof(double) * (size_t)S->n);
}

void orc_get_stress(const orc_state *S, double out[27]) { memcpy(out, S->stress, sizeof(S->stress)); }

/* Five 3x3 stresses of the last evaluation: contact (with the repulsion),
 * lubrication, instantaneous Brownian, drag stresslet, and the total of Sec.
 * IV.D, hydrodynamic (lubrication + drag) plus contact; the Brownian stress
 * averages to zero and is not part of the total. */
void orc_get_stress_all(const orc_state *S, double out[45])
{
    memcpy(out, S->stress, sizeof(S->stress));
    memcpy(out + 27, S->drag, sizeof(S->drag));
    for (int k = 0; k < 9; ++k) out[36 + k] = S->stress[k] + S->stress[9 + k] + S->drag[k];
}

/* Relative viscosity of the last evaluation, Sec. II.E: Sigma_xy / (eta gammadot)
 * of the total stress (NaN without shear). */
double orc_eta_r(const orc_state *S)
{
    double t = S->stress[1] + S->stress[9 + 1] + S->drag[1];
    return t / (S->p.eta * S->p.gammadot);
}

/* Time autocorrelation of a per-step series, the integrand of the Green-Kubo
 * integral of Sec. IV.B: out[k] = mean over t of s(t) s(t + k), for k < nlag,
 * over the count - k available pairs of records (0 where none). */
void orc_acf(const double *s, long count, long nlag, double *out)
{
    for (long k = 0; k < nlag; ++k) {
        double acc = 0.0;
        for (long t = 0; t + k < count; ++t) acc += s[t] * s[t + k];
        out[k] = k < count ? acc / (double)(count - k) : 0.0;
    }
}

void orc_get_disp(const orc_state *S, double *out_3n) { memcpy(out_3n, S->disp, sizeof(double) * 3 * (size_t)S->n); }

/* Histogram of pair distances r < r_max (each pair once, minimum image in the sheared
   box), bins of width r_max / nbins; brute force over all pairs. */
void orc_rdf(const orc_state *S, double r_max, int nbins, uint64_t *counts)
{
    for (int k = 0; k < nbins; ++k) counts[k] = 0;
    for (int i = 0; i < S->n; ++i)
        for (int j = i + 1; j < S->n; ++j) {
            double r[3];
            min_image(&S->p, S->s_le, &S->x[3 * i], &S->x[3 * j], r);
            double d = sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
            if (!(d < r_max)) continue;
            int k = (int)(d / r_max * (double)nbins);
            if (k >= nbins) k = nbins - 1;
            counts[k] += 1;
        }
}

/* Slice of the pair distribution through the flow-gradient plane (Sec. IV.D):
   pairs with |r_z| < slab/2 and |r_x|, |r_y| < r_max, counted at r and at -r on
   an nbins x nbins grid over [-r_max, r_max)^2 (counts[ix * nbins + iy]);
   brute force over all pairs, minimum image in the sheared box. */
void orc_rdf_xy(const orc_state *S, double r_max, double slab, int nbins, uint64_t *counts)
{
    for (long k = 0; k < (long)nbins * nbins; ++k) counts[k] = 0;
    for (int i = 0; i < S->n; ++i)
        for (int j = i + 1; j < S->n; ++j) {
            double r[3];
            min_image(&S->p, S->s_le, &S->x[3 * i], &S->x[3 * j], r);
            if (!(fabs(r[2]) < 0.5 * slab) || !(fabs(r[0]) < r_max) || !(fabs(r[1]) < r_max)) continue;
            for (int sgn = 0; sgn < 2; ++sgn) {
                double ux = sgn ? -r[0] : r[0], uy = sgn ? -r[1] : r[1];
                int ix = (int)((ux + r_max) / (2.0 * r_max) * (double)nbins);
                int iy = (int)((uy + r_max) / (2.0 * r_max) * (double)nbins);
                if (ix >= nbins) ix = nbins - 1;
                if (iy >= nbins) iy = nbins - 1;
                counts[(long)ix * nbins + iy] += 1;
            }
        }
}

/* Runs nsteps steps and adds the pair-distance histogram of the configuration
   after every `every`-th step to counts (the g(r) sampling of Sec. III.A). */
void orc_run_rdf(orc_state *S, long nsteps, long every, double r_max, int nbins, uint64_t *counts)
{
    uint64_t *c = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nbins);
    for (long t = 1; t <= nsteps; ++t) {
        step(S);
        if (t % every) continue;
        orc_rdf(S, r_max, nbins, c);
        for (int k = 0; k < nbins; ++k) counts[k] += c[k];
    }
    free(c);
}

/* Structural Brownian stress of the current configuration, Sec. II.D:
   -(kT/V) sum_i (a_i/Delta_i) sum_{j: h_ij <= Delta_i} n_ij (x) n_ij with
   Delta_i = 0.05 a_i and h_ij = |r_ij| - (a_i + a_j); all pairs, brute force. */
void orc_structural_stress(const orc_state *S, double out[9])
{
    const orc_params *p = &S->p;
    double acc[9] = {0};
    for (int i = 0; i < S->n; ++i)
        for (int j = 0; j < S->n; ++j) {
            if (j == i) continue;
            double r[3];
            min_image(p, S->s_le, &S->x[3 * i], &S->x[3 * j], r);
            double dist = sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
            double h = dist - (S->a[i] + S->a[j]);
            double delta = 0.05 * S->a[i];
            if (!(h <= delta)) continue;
            double wgt = S->a[i] / delta;
            for (int al = 0; al < 3; ++al)
                for (int be = 0; be < 3; ++be) acc[3 * al + be] += wgt * (r[al] / dist) * (r[be] / dist);
        }
    double V = p->L[0] * p->L[1] * p->L[2];
    for (int k = 0; k < 9; ++k) out[k] = -p->kT / V * acc[k];
}

/* Contacts (sorted by (i, j)); returns the count, fills at most cap. */
int orc_get_contacts(const orc_state *S, int cap, uint32_t *ij, double *s, int32_t *sliding)
{
    for (int q = 0; q < S->nc && q < cap; ++q) {
        ij[2 * q] = S->c[q].i; ij[2 * q + 1] = S->c[q].j;
        s[3 * q] = S->c[q].s[0]; s[3 * q + 1] = S->c[q].s[1]; s[3 * q + 2] = S->c[q].s[2];
        if (sliding) sliding[q] = S->c[q].sliding;
    }
    return S->nc;
}

/* Interaction set of the last evaluation (pairs with xi <= xi_cut), sorted. */
int orc_get_pairs(const orc_state *S, int cap, uint32_t *ij)
{
    for (int q = 0; q < S->npairs && q < cap; ++q) { ij[2 * q] = S->pairs[2 * q]; ij[2 * q + 1] = S->pairs[2 * q + 1]; }
    return S->npairs;
}

/* Verlet set at the current positions: all pairs with
 * |r| <= (a_i + a_j)(1 + xi_cut/2) + skin, brute force, sorted. */
long orc_verlet_pairs(const orc_state *S, double skin, long cap, uint32_t *ij)
{
    long cnt = 0;
    double c1 = 1.0 + 0.5 * S->p.xi_cut;
    for (int i = 0; i < S->n; ++i)
        for (int j = i + 1; j < S->n; ++j) {
            double r[3];
            min_image(&S->p, S->s_le, &S->x[3 * i], &S->x[3 * j], r);
            double d2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
            double rl = (S->a[i] + S->a[j]) * c1 + skin;
            if (d2 <= rl * rl) {
                if (cnt < cap) { ij[2 * cnt] = (uint32_t)i; ij[2 * cnt + 1] = (uint32_t)j; }
                cnt++;
            }
        }
    return cnt;
}

/* Force and torque on a single particle i, computed by visiting every other
 * particle (O(N) per call), for spot checks of very large systems.  Uses the
 * stored contact history; nothing in the state is modified.  F, T: 3 doubles.
 * Also returns the norm sums used to normalise errors. */
void orc_particle_force(orc_state *S, int i, double F[3], double T[3], double *Fabs, double *Tabs)
{
    /* evaluate on a scratch copy of the accumulators */
    double *Fs = S->F, *Ts = S->T, *Fa = S->Fabs, *Ta = S->Tabs;
    double st[27];
    memcpy(st, S->stress, sizeof(st));
    int np = S->npairs;
    size_t n = (size_t)S->n;
    S->F = (double *)calloc(3 * n, sizeof(double));
    S->T = (double *)calloc(3 * n, sizeof(double));
    S->Fabs = (double *)calloc(n, sizeof(double));
    S->Tabs = (double *)calloc(n, sizeof(double));
    contact_io io = {NULL, 0, 0, S->c, S->nc, 0};
    for (int j = 0; j < S->n; ++j) {
        if (j == i) continue;
        if (i < j) pair_force(S, i, j, &io); else pair_force(S, j, i, &io);
    }
    if (!(S->p.flags & ORC_NO_ONEBODY)) {
        const orc_params *p = &S->p;
        double b = sqrt(2.0 * p->kT / p->dt);
        double zeta = 6.0 * ORC_PI * p->eta * S->a[i];
        double zr = 8.0 * ORC_PI * p->eta * S->a[i] * S->a[i] * S->a[i];
        double Uinf[3] = {p->gammadot * (S->x[3 * i + 1] - 0.5 * p->L[1]), 0.0, 0.0};
        double Oinf[3] = {0.0, 0.0, -0.5 * p->gammadot};
        double psi[3], phi[3];
        gauss_one(p, S->k, (uint32_t)i, ORC_STREAM_ONE_FORCE, psi);
        gauss_one(p, S->k, (uint32_t)i, ORC_STREAM_ONE_TORQUE, phi);
        double sz = sqrt(zeta), szr = sqrt(zr);
        double fd[3], td[3];
        for (int d = 0; d < 3; ++d) {
            fd[d] = zeta * (Uinf[d] - S->v[3 * i + d]) + b * sz * psi[d];
            td[d] = zr * (Oinf[d] - S->w[3 * i + d]) + b * szr * phi[d];
            S->F[3 * i + d] += fd[d];
            S->T[3 * i + d] += td[d];
        }
        S->Fabs[i] += norm3(fd);
        S->Tabs[i] += norm3(td);
    }
    for (int d = 0; d < 3; ++d) { F[d] = S->F[3 * i + d]; T[d] = S->T[3 * i + d]; }
    *Fabs = S->Fabs[i]; *Tabs = S->Tabs[i];
    free(S->F); free(S->T); free(S->Fabs); free(S->Tabs); free(io.cnew);
    S->F = Fs; S->T = Ts; S->Fabs = Fa; S->Tabs = Ta;
    memcpy(S->stress, st, sizeof(st));
    S->npairs = np;
}
