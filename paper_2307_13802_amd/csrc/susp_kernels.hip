// gfx950 kernels of the sheared-suspension force engine.
//
// A time step is two launches over all replicas: integrate (kick 1, drift,
// Lees-Edwards wrap, bound on the displacement since the last list build,
// list-expiry test) and pair force (all pair and one-body terms, kick 2,
// stress with a fixed-order reduction, advance of the step counter).  The
// cell/list rebuild (Hilbert-ordered cell keys, scan, scatter, in-cell ordering,
// reorder, Verlet list with contact-history carry-over) is launched by the
// host only when its displacement budget is used up, or when the expiry test
// halted a step.  Paper references are to Li, Royer & Ness, arXiv 2307.13802.
//
// Compiled with -ffp-contract=off: the geometry, the neighbour predicate and
// the contact-history update are evaluated operation by operation in the
// same order as the plain FP64 definition, so neighbour sets and springs are
// bit-reproducible; FP64 division and square root are IEEE correctly rounded.
#include <hip/hip_ext.h>

#include <mutex>
#include <string>

#include "susp.h"

namespace susp {

// ---------------------------------------------------------------------------
// Counter-based noise: Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw,
// SC'11), Box-Muller normals.  Counter words: (step_lo, id_a, id_b,
// step_hi << 8 | stream); stream 0 = pair force (id_a < id_b), 2 and 3 =
// one-body force and torque (id_b = 0xFFFFFFFF).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ void normals3(uint4 w, double g[3]) {
    const double s = 2.3283064365386963e-10;  // 2^-32
    const double u0 = ((double)w.x + 0.5) * s, u1 = ((double)w.y + 0.5) * s;
    const double u2 = ((double)w.z + 0.5) * s, u3 = ((double)w.w + 0.5) * s;
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    double s1, c1;
    sincospi(2.0 * u1, &s1, &c1);  // sin, cos of 2 pi u1 (the doubling is exact)
    g[0] = r0 * c1;
    g[1] = r0 * s1;
    g[2] = r1 * cospi(2.0 * u3);
}

__device__ __forceinline__ void normals3(uint4 w, float g[3]) {
    const float s = 2.3283064365386963e-10f;
    const float u0 = ((float)w.x + 0.5f) * s, u1 = ((float)w.y + 0.5f) * s;
    const float u2 = ((float)w.z + 0.5f) * s, u3 = ((float)w.w + 0.5f) * s;
    // hardware log2 and sin/cos of 2*pi*x (argument in revolutions)
    const float r0 = __builtin_amdgcn_sqrtf(-2.0f * 0.69314718055994531f * __builtin_amdgcn_logf(u0));
    const float r1 = __builtin_amdgcn_sqrtf(-2.0f * 0.69314718055994531f * __builtin_amdgcn_logf(u2));
    g[0] = r0 * __builtin_amdgcn_cosf(u1);
    g[1] = r0 * __builtin_amdgcn_sinf(u1);
    g[2] = r1 * __builtin_amdgcn_cosf(u3);
}

// ---------------------------------------------------------------------------
// Geometry in the sheared periodic box (Sec. II.E as a Lees-Edwards offset s:
// the image of a particle shifted by +Ly in y is shifted by +s in x).
// d = x_a - x_b over the nearest image; returns k_y, the number of Ly periods
// between a and the image of b.  Pairs within the interaction range are far
// from the half-box points where the rounding of t/L could matter.
// ---------------------------------------------------------------------------
// (t * (1/L) rounds to the same integer as t / L except within an ulp of a
// half-integer, i.e. for separations of half a box, far outside any list range.)
__device__ __forceinline__ int min_image(const double* L, const double* invL, double s_le, const double4& pa,
                                         const double4& pb, double& dx, double& dy, double& dz) {
    dy = pa.y - pb.y;
    const double ky = rint(dy * invL[1]);
    dy = dy - ky * L[1];
    dx = (pa.x - pb.x) - ky * s_le;
    dx = dx - L[0] * rint(dx * invL[0]);
    dz = pa.z - pb.z;
    dz = dz - L[2] * rint(dz * invL[2]);
    return (int)ky;
}
__device__ __forceinline__ int min_image(const RepParams& P, double s_le, const double4& pa, const double4& pb,
                                         double& dx, double& dy, double& dz) {
    return min_image(P.L, P.invL, s_le, pa, pb, dx, dy, dz);
}

__device__ __forceinline__ uint32_t part1by2(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Cell key along a 3D Hilbert curve over [0, 2^b)^3 (J. Skilling, "Programming the
// Hilbert curve", AIP Conf. Proc. 707 (2004): the coordinates are transformed in place,
// then their bits interleaved, the first coordinate most significant).  Consecutive keys
// are face neighbours, so particles in key order keep their neighbours near in memory
// (without the long jumps of Morton order at its block boundaries).
__device__ __forceinline__ uint32_t hilbert3(uint32_t x, uint32_t y, uint32_t z, int b) {
    if (b == 0) return 0u;
    uint32_t X[3] = {x, y, z};
    const uint32_t M = 1u << (b - 1);
    for (uint32_t Q = M; Q > 1u; Q >>= 1) {   // undo excess work
        const uint32_t P = Q - 1u;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;   // invert the low bits of the first
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;   // exchange the low bits
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];   // Gray encode
    X[2] ^= X[1];
    uint32_t t = 0u;
    for (uint32_t Q = M; Q > 1u; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1u;
    X[0] ^= t;
    X[1] ^= t;
    X[2] ^= t;
    return part1by2(X[2]) | (part1by2(X[1]) << 1) | (part1by2(X[0]) << 2);
}

__device__ __forceinline__ uint32_t cell_key(const RepParams& P, int x, int y, int z) {
    return P.key_off + hilbert3((uint32_t)x, (uint32_t)y, (uint32_t)z, P.mbits);
}

__device__ __forceinline__ int cell_coord(double x, double w, int n) {
    int c = (int)floor(x / w);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

__device__ __forceinline__ float as_posf(uint32_t b) { return __uint_as_float(b); }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Particle kernels map block b to tile xcd_tile(b, g) so that every XCD
// walks one contiguous range of Hilbert-ordered tiles: neighbours' data then
// sits in the L2 of the XCD that reads it.  A bijection of [0, g).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t g) {
    const uint32_t x = b & 7u, k = b >> 3, per = g >> 3, rem = g & 7u;
    return x * per + (x < rem ? x : rem) + k;
}
// The same ranges walked from their ends: the gather, which follows the pair kernel,
// starts where that kernel finished, so the pair records and particle data it wrote
// last are still in the XCD's L2 (and the next pair kernel starts where the gather
// finished).  A bijection of [0, g): block b's position k in its XCD's range is below
// that range's length.
__device__ __forceinline__ uint32_t xcd_tile_rev(uint32_t b, uint32_t g) {
    const uint32_t x = b & 7u, k = b >> 3, per = g >> 3, rem = g & 7u;
    const uint32_t len = per + (x < rem ? 1u : 0u);
    return x * per + (x < rem ? x : rem) + (len - 1u - k);
}

// Lees-Edwards offset one step after the stored one (same arithmetic everywhere)
__device__ __forceinline__ double next_offset(const RepParams& P, double s_le) {
    double s = s_le + P.gdLy * P.dt;
    return s - P.L[0] * floor(s / P.L[0]);
}

// Cross-lane moves on the DPP network (no LDS traffic).  CTRL: 0x111..0x118 =
// row_shr:1..8 (lanes past the row edge read 0), 0xB1 / 0x4E = quad_perm swaps
// of neighbouring lanes / lane pairs.
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL> __device__ __forceinline__ unsigned long long dpp_u64(unsigned long long u) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, true);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
template <int CTRL> __device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Pair records in memory: three doubles (24 B) in FP64; a float4 in mixed
// precision, so that one aligned access moves it.
struct Rec3d {
    double x, y, z;
};
template <class R> struct PairRec;
template <> struct PairRec<double> {
    using T = Rec3d;
    static __device__ __forceinline__ T make(double a, double b, double c) { return Rec3d{a, b, c}; }
};
template <> struct PairRec<float> {
    using T = float4;
    static __device__ __forceinline__ T make(float a, float b, float c) { return make_float4(a, b, c, 0.0f); }
};

// spring of list entry slot k (k = e * npad + i): three components, packed
template <class R> struct Spring {
    R x, y, z;
};
template <class R> __device__ __forceinline__ void load_spring(const Bufs& b, uint32_t k, R* s) {
    const Spring<R> v = ((const Spring<R>*)b.hs)[k];
    s[0] = v.x; s[1] = v.y; s[2] = v.z;
}
template <class R> __device__ __forceinline__ void store_spring(const Bufs& b, uint32_t k, const R* s) {
    ((Spring<R>*)b.hs)[k] = Spring<R>{s[0], s[1], s[2]};
}
// non-temporal double4 access (one access, not kept in the L2), for data that no kernel
// reads soon after
typedef double nt_d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double4 ld_nt(const double4* p) {
    const nt_d4 v = __builtin_nontemporal_load((const nt_d4*)p);
    return make_double4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_nt(double4* p, const double4& v) {
    const nt_d4 t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, (nt_d4*)p);
}
// the pair kernel's read of a stored spring: once per step, so not kept in the L2
template <class R> __device__ __forceinline__ void load_spring_nt(const Bufs& b, uint32_t k, R* s) {
    const R* p = (const R*)((const Spring<R>*)b.hs + k);
    s[0] = __builtin_nontemporal_load(p);
    s[1] = __builtin_nontemporal_load(p + 1);
    s[2] = __builtin_nontemporal_load(p + 2);
}
// the pair kernel's spring update: read again only by the next step's pair kernel, so
// stored past the L2 (non-temporal), which keeps the L2 for the records the gather reads
template <class R> __device__ __forceinline__ void store_spring_nt(const Bufs& b, uint32_t k, const R* s) {
    R* p = (R*)((Spring<R>*)b.hs + k);
    __builtin_nontemporal_store(s[0], p);
    __builtin_nontemporal_store(s[1], p + 1);
    __builtin_nontemporal_store(s[2], p + 2);
}
// in FP64 whatever the precision of the handle (rebuild carry, diagnostics)
__device__ __forceinline__ void spring_f64(const Bufs& b, uint32_t k, double* s) {
    if (b.mixed) {
        float t[3];
        load_spring<float>(b, k, t);
        s[0] = t[0]; s[1] = t[1]; s[2] = t[2];
    } else {
        load_spring<double>(b, k, s);
    }
}

// inclusive sum over each 16-lane row; lane 15 of a row then holds the row total
__device__ __forceinline__ double row_sum_f64(double x) {
    x += dpp_f64<0x111>(x);
    x += dpp_f64<0x112>(x);
    x += dpp_f64<0x114>(x);
    x += dpp_f64<0x118>(x);
    return x;
}

// block-wide max of a non-negative float, stored by thread 0
__device__ __forceinline__ void block_max_store(float v, float* out) {
    __shared__ float rows[16];
    v = fmaxf(v, dpp_f32<0x111>(v));
    v = fmaxf(v, dpp_f32<0x112>(v));
    v = fmaxf(v, dpp_f32<0x114>(v));
    v = fmaxf(v, dpp_f32<0x118>(v));
    if ((threadIdx.x & 15) == 15) rows[threadIdx.x >> 4] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = rows[0];
        for (int k = 1; k < (int)(blockDim.x >> 4); ++k) m = fmaxf(m, rows[k]);
        *out = m;
    }
}

// Reduction of one stress component c of replica r from the partials of
// parity x, in a fixed order (one block), unless already done; component 0
// also checks the overlap limit.
__device__ void finalize_unit(const Bufs& b, uint32_t r, int c, int x) {
    RepDyn& D = b.dyn[r];
    const uint32_t id = D.eval_id[x];
    if (id == D.done_id[x][c]) return;  // uniform across the block
    const RepParams& P = b.reps[r];
    const uint32_t blk0 = P.p_begin / (uint32_t)b.ppb, nblk = P.n_pad / (uint32_t)b.ppb;
    const double* part = b.partial + ((size_t)x * 27 + c) * b.nblk_max + blk0;
    double v = 0.0;
    for (uint32_t k = threadIdx.x; k < nblk; k += blockDim.x) v += part[k];
    __shared__ double rows[16];
    __shared__ float mrows[16];
    v = row_sum_f64(v);
    if ((threadIdx.x & 15) == 15) rows[threadIdx.x >> 4] = v;
    if (c == 0) {  // largest overlap of the evaluation, from the block maxima
        const float* op = b.ovpart + (size_t)x * b.nblk_max + blk0;
        float m = 0.0f;
        for (uint32_t k = threadIdx.x; k < nblk; k += blockDim.x) m = fmaxf(m, op[k]);
        m = fmaxf(m, dpp_f32<0x111>(m));
        m = fmaxf(m, dpp_f32<0x112>(m));
        m = fmaxf(m, dpp_f32<0x114>(m));
        m = fmaxf(m, dpp_f32<0x118>(m));
        if ((threadIdx.x & 15) == 15) mrows[threadIdx.x >> 4] = m;
    }
    __syncthreads();
    __shared__ double total;
    const uint32_t rec = D.rec[x];
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 4); ++k) t += rows[k];
        total = t;
        b.last[r * 27 + c] = t;
        if (rec) {
            b.ring[((size_t)r * kRing + (rec - 1) % kRing) * 27 + c] = t;
            D.stress_sum[c] += t;
        }
        if (c == 0) {
            float mo = 0.0f;
            for (int k = 0; k < (int)(blockDim.x >> 4); ++k) mo = fmaxf(mo, mrows[k]);
            if ((double)mo > P.max_overlap) D.health |= H_OVERLAP;
            D.maxov_last_bits = __float_as_uint(mo);
        }
        D.done_id[x][c] = id;
    }
    __syncthreads();
    if (rec && c == b.acf_comp) {
        // streaming autocorrelation: each lag's sum gains s(t) s(t - k), one thread per lag,
        // the terms of every lag in time order
        const uint32_t W = b.acf_nlag;
        const unsigned long long ns = b.acf_n[r];
        double* hist = b.acf_hist + (size_t)r * W;
        double* sum = b.acf_sum + (size_t)r * W;
        const double v = total;
        for (uint32_t k = threadIdx.x; k < W && (unsigned long long)k <= ns; k += blockDim.x)
            sum[k] += (k == 0 ? v : hist[(ns - k) % W]) * v;
        __syncthreads();
        if (threadIdx.x == 0) {
            hist[ns % W] = v;
            b.acf_n[r] = ns + 1;
        }
        __syncthreads();
    }
}

// units (replica, component) handled by the blocks of a grid, in turn
__device__ void finalize_all(const Bufs& b, int x) {
    for (uint32_t u = blockIdx.x; u < 27u * b.nrep; u += gridDim.x) finalize_unit(b, u / 27u, (int)(u % 27u), x);
}

__global__ __launch_bounds__(256) void k_finalize(Bufs b, int x) { finalize_all(b, x); }

// ---------------------------------------------------------------------------
// List validity.  A pair outside the list at the last build (|r| > r_c +
// skin) can have come within r_c by time t only if 2 D + |gammadot| t (r_c +
// 4 D) > skin, where D = max(d_i, d_j), d_i bounds particle i's non-affine
// displacement since the build (drift minus the imposed flow integrated
// along the path) and t is the time since the build: the affine part of the
// relative motion is gammadot r_y t along x, with |r_y| <= r_c + 4 D over the
// interval.  With 2 D <= skin this is implied by 2 D + |gammadot| t (r_c +
// 2 skin) > skin, so each particle tests its own bound after its drift; one
// failure flags the step (expire), its force launch does nothing and the
// host rebuilds the lists from the moved positions before evaluating it.
// ---------------------------------------------------------------------------
// (rcs = r_c + 2 skin, with r_c the largest interaction range)
__device__ __forceinline__ bool list_expired(double gd, double rcs, double skin, double d, double t) {
    return 2.0 * d + fabs(gd) * t * rcs > skin;
}

// ---------------------------------------------------------------------------
// Kick 1, drift and wrap of a step with parity q (velocity-Verlet, Sec. II;
// sheared box, Sec. II.E).  Also accumulates each particle's non-affine
// displacement |dx - U^inf dt| and applies the list-validity test.
// ---------------------------------------------------------------------------
// What kick 1, the drift, the wrap and the validity test of the step with parity q
// read of the replica's parameters and bookkeeping.  Kernels read it before their
// first store: the compiler cannot tell that those stores leave it unchanged, and
// would otherwise read each value again after them (a memory round trip at the end
// of every lane's work).
struct DriftPar {
    double L[3], gd, gdLy, dt, half_dt, rho, skin, rcs, s_next, t_next;
    uint32_t flags;
};
__device__ __forceinline__ DriftPar drift_par(const RepParams& P, const RepDyn& D, int q) {
    DriftPar d;
    for (int k = 0; k < 3; ++k) d.L[k] = P.L[k];
    d.gd = P.gd;
    d.gdLy = P.gdLy;
    d.dt = P.dt;
    d.half_dt = P.half_dt;
    d.rho = P.rho;
    d.skin = P.skin;
    d.rcs = P.rc_max + 2.0 * P.skin;
    d.s_next = next_offset(P, D.s_slot[1 - q]);
    d.t_next = D.t_slot[1 - q] + P.dt;
    d.flags = P.flags;
    return d;
}

// one half kick of velocity-Verlet: v += dt/2 F / m, w += dt/2 T / I
__device__ __forceinline__ void half_kick(double a, double rho, double half_dt, const double* F, const double* T,
                                          double4& v, double4& w) {
    const double m = (4.0 / 3.0) * kPi * rho * a * a * a;
    const double I = 0.4 * m * a * a;
    const double hm = half_dt / m, hI = half_dt / I;
    v.x += hm * F[0]; v.y += hm * F[1]; v.z += hm * F[2];
    w.x += hI * T[0]; w.y += hI * T[1]; w.z += hI * T[2];
}

// Kick 1, drift and wrap of particle i (parameters dp of the step), from its
// full-step velocities v, w, position x and the force and torque F, T of the
// last evaluation (as stored); da, dacc: its displacement records as read (da only
// with F_TRACK_DISP);
// accumulates its displacement bound (dblk) and applies the list-validity test
// (expire).
template <bool MIX>
__device__ __forceinline__ void integrate_particle(const Bufs& b, const DriftPar& dp, uint32_t i, double4 x,
                                                   double4 v, double4 w, const double* F, const double* T,
                                                   double4 da, double dacc, float& dblk, bool& expire) {
    double disp = 0.0;
    half_kick(x.w, dp.rho, dp.half_dt, F, T, v, w);
    if (!(dp.flags & F_FREEZE_X)) {
        const double yold = x.y;
        const double vdx = v.x, vdy = v.y, vdz = v.z;  // drift velocity
        x.x += dp.dt * v.x;
        x.y += dp.dt * v.y;
        x.z += dp.dt * v.z;
        const double s = dp.s_next;
        const double Lx = dp.L[0], Ly = dp.L[1], Lz = dp.L[2];
        if (x.y >= Ly) {
            x.y -= Ly; x.x -= s; v.x -= dp.gdLy;
        } else if (x.y < 0.0) {
            x.y += Ly; x.x += s; v.x += dp.gdLy;
            if (x.y >= Ly) x.y = 0.0;
        }
        x.x -= Lx * floor(x.x / Lx);
        x.z -= Lz * floor(x.z / Lz);
        if (x.x >= Lx) x.x -= Lx;
        if (x.z >= Lz) x.z -= Lz;
        // non-affine displacement of this step: drift minus the imposed flow
        // integrated along the path, gammadot (y(t) - Ly/2) with y(t) = yold + vdy t
        const double ux = dp.gd * (yold - 0.5 * Ly) + 0.5 * dp.gd * dp.dt * vdy;
        const double ex = dp.dt * (vdx - ux), ey = dp.dt * vdy, ez = dp.dt * vdz;
        disp = sqrt(ex * ex + ey * ey + ez * ez) * (1.0 + 1e-6) + 1e-30;
        b.pos[i] = x;
        if (dp.flags & F_TRACK_DISP) {
            da.x += ex; da.y += ey; da.z += ez;
            b.disp[i] = da;
        }
    }
    if (MIX) {   // only the next step's gather reads the FP64 half-step velocities: past the L2
        st_nt(&b.vh[i], v);
        st_nt(&b.wh[i], w);
    } else {
        b.vh[i] = v;
        b.wh[i] = w;
    }
    if (MIX) {
        b.vsh[i] = make_float4((float)v.x, (float)v.y, (float)v.z, 0.0f);
        b.wsh[i] = make_float4((float)w.x, (float)w.y, (float)w.z, 0.0f);
    }
    const double d = dacc + disp;
    // rounded up: the stored bound stays a bound; read again only by the next step's
    // integrate, so stored past the L2
    __builtin_nontemporal_store(__double2float_ru(d), &b.dacc[i]);
    expire = list_expired(dp.gd, dp.rcs, dp.skin, d, dp.t_next);
    dblk = (float)d * (1.0f + 1e-6f);
}

template <bool MIX>
__global__ __launch_bounds__(256) void k_integrate(Bufs b, int q) {
    if (b.sys->halted) return;  // uniform: set by an earlier launch
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t i = tile * blockDim.x + threadIdx.x;
    // replicas are padded to whole tiles, so r is uniform over a block (here and in
    // every kernel): readfirstlane keeps it, and what derives from it, scalar
    const uint32_t r = __builtin_amdgcn_readfirstlane(b.blk_rep[i / kTile]);
    const RepParams& P = b.reps[r];
    const RepDyn& D = b.dyn[r];
    const DriftPar dp = drift_par(P, D, q);
    float dblk = 0.0f;
    bool expire = false;
    if (i - P.p_begin < P.n) {
        double F[3], T[3];
        if (MIX) {
            const float4 f = ((const float4*)b.F)[i], t = ((const float4*)b.T)[i];
            F[0] = f.x; F[1] = f.y; F[2] = f.z; T[0] = t.x; T[1] = t.y; T[2] = t.z;
        } else {
            const double4 f = ((const double4*)b.F)[i], t = ((const double4*)b.T)[i];
            F[0] = f.x; F[1] = f.y; F[2] = f.z; T[0] = t.x; T[1] = t.y; T[2] = t.z;
        }
        const double4 da = (dp.flags & F_TRACK_DISP) ? b.disp[i] : make_double4(0.0, 0.0, 0.0, 0.0);
        integrate_particle<MIX>(b, dp, i, b.pos[i], b.vf[i], b.wf[i], F, T, da, b.dacc[i], dblk, expire);
    }
    if (expire) atomicOr(&b.sys->expire[q], 1u);  // rare: the lists are rebuilt before that
    block_max_store(dblk, &b.dpart[(size_t)q * (b.npad / kTile) + tile]);
}

// ---------------------------------------------------------------------------
// Rebuild: Hilbert-ordered cells, deterministic order inside a cell (by id),
// reorder of all particle data, neighbour list with history carry-over.
// ---------------------------------------------------------------------------
__global__ void k_rb_zero(Bufs b) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < b.nkeys_total) {
        b.cell_cnt[k] = 0u;
        b.cell_fill[k] = 0u;
    }
}

__global__ __launch_bounds__(256) void k_rb_keys(Bufs b) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t r = __builtin_amdgcn_readfirstlane(b.blk_rep[q / kTile]);
    const RepParams& P = b.reps[r];
    const uint32_t lq = q - P.p_begin;
    if (lq < P.n) {
        const double4 x = b.pos[q];
        const int cx = cell_coord(x.x, P.cw[0], P.nc[0]);
        const int cy = cell_coord(x.y, P.cw[1], P.nc[1]);
        const int cz = cell_coord(x.z, P.cw[2], P.nc[2]);
        const uint32_t key = cell_key(P, cx, cy, cz);
        b.key[q] = key;
        atomicAdd(&b.cell_cnt[key], 1u);
    } else if (lq == P.n && P.n_pad > P.n) {
        // the padding slots of the replica form one extra cell at its end
        atomicAdd(&b.cell_cnt[P.key_off + P.nkeys - 1], P.n_pad - P.n);
    }
}

// exclusive scan of cell counts: per-block sums, scan of the sums, down-sweep
constexpr int kScanPer = 4;
constexpr int kScanBlock = 256;
constexpr int kScanTile = kScanPer * kScanBlock;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wsum[kScanBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) {
        if (w < wave) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(Bufs b) {
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    uint32_t s = 0;
#pragma unroll
    for (int t = 0; t < kScanPer; ++t) s += (base + t < b.nkeys_total) ? b.cell_cnt[base + t] : 0u;
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) b.scan_blk[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_top(Bufs b, uint32_t nblk) {
    // single block: scan nblk block sums in chunks of kScanBlock
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < nblk; c0 += kScanBlock) {
        const uint32_t k = c0 + threadIdx.x;
        const uint32_t v = k < nblk ? b.scan_blk[k] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, &tot);
        if (k < nblk) b.scan_blk[k] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) b.cell_start[b.nkeys_total] = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_down(Bufs b) {
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t s = 0;
#pragma unroll
    for (int t = 0; t < kScanPer; ++t) {
        v[t] = (base + t < b.nkeys_total) ? b.cell_cnt[base + t] : 0u;
        s += v[t];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(s, &tot) + b.scan_blk[blockIdx.x];
#pragma unroll
    for (int t = 0; t < kScanPer; ++t) {
        if (base + t < b.nkeys_total) b.cell_start[base + t] = ex;
        ex += v[t];
    }
}

__global__ __launch_bounds__(256) void k_rb_scatter(Bufs b) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t r = __builtin_amdgcn_readfirstlane(b.blk_rep[q / kTile]);
    const RepParams& P = b.reps[r];
    if (q - P.p_begin < P.n) {
        const uint32_t key = b.key[q];
        const uint32_t slot = b.cell_start[key] + atomicAdd(&b.cell_fill[key], 1u);
        b.src[slot] = q;
    }
}

// order the members of each cell by particle id (makes the layout independent of atomic order)
__global__ void k_rb_cellsort(Bufs b) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.nkeys_total) return;
    const uint32_t cnt = b.cell_fill[k];
    if (cnt < 2 || cnt != b.cell_cnt[k]) return;  // padding cells have fill 0
    const uint32_t s0 = b.cell_start[k];
    for (uint32_t a = 1; a < cnt; ++a) {
        const uint32_t v = b.src[s0 + a];
        const uint32_t idv = b.id[v];
        int c = (int)a - 1;
        while (c >= 0 && b.id[b.src[s0 + c]] > idv) {
            b.src[s0 + c + 1] = b.src[s0 + c];
            --c;
        }
        b.src[s0 + c + 1] = v;
    }
}

// gather every particle array into its new slot (staging copies), and turn
// the per-entry contact history of the old list into a compact per-particle
// table keyed by partner id
__global__ __launch_bounds__(256) void k_rb_gather(Bufs b, uint32_t ct_input_rep) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t r = __builtin_amdgcn_readfirstlane(b.blk_rep[q / kTile]);
    const RepParams& P = b.reps[r];
    const uint32_t npad = b.npad;
    if (q - P.p_begin >= P.n) {
        b.alt_id[q] = kNoId;
        for (int a = 0; a < 8; ++a) b.alt4[a][q] = make_double4(0.0, 0.0, 0.0, 0.0);
        b.ct_n[q] = 0u;
        return;
    }
    const uint32_t s = b.src[q];
    b.alt_id[q] = b.id[s];
    b.alt4[0][q] = b.pos[s];
    b.alt4[1][q] = b.vh[s];
    b.alt4[2][q] = b.wh[s];
    b.alt4[3][q] = b.vf[s];
    b.alt4[4][q] = b.wf[s];
    b.alt4[7][q] = b.disp[s];
    if (b.mixed) {
        const float4 f = ((const float4*)b.F)[s], t = ((const float4*)b.T)[s];
        b.alt4[5][q] = make_double4(f.x, f.y, f.z, 0.0);
        b.alt4[6][q] = make_double4(t.x, t.y, t.z, 0.0);
    } else {
        b.alt4[5][q] = ((const double4*)b.F)[s];
        b.alt4[6][q] = ((const double4*)b.T)[s];
    }
    uint32_t c = 0;
    if (ct_input_rep == 0xFFFFFFFEu || r == ct_input_rep) {
        // history given by the host in compact form at the old slot (second table)
        const uint32_t nin = b.ct_n[npad + s];
        for (uint32_t e = 0; e < nin && c < (uint32_t)kCtCap; ++e, ++c) {
            b.ct_id[c * npad + q] = b.ct_id[(kCtCap + e) * npad + s];
            for (int d = 0; d < 3; ++d) b.ct_s[(c * 3 + d) * npad + q] = b.ct_s[((kCtCap + e) * 3 + d) * npad + s];
            b.ct_sl[c * npad + q] = 0;
        }
    } else {
        const uint64_t cm = b.cmask[s], sm = b.smask[s];
        const uint32_t cnt = b.ncnt[s];
        for (uint32_t e = 0; e < cnt; ++e) {
            if (!((cm >> e) & 1ull)) continue;
            if (c >= (uint32_t)kCtCap) {
                atomicOr(&b.dyn[r].health, H_NLIST);
                break;
            }
            b.ct_id[c * npad + q] = b.id[b.nbr[e * npad + s]];
            double hv[3];
            spring_f64(b, e * npad + s, hv);
            for (int d = 0; d < 3; ++d) b.ct_s[(c * 3 + d) * npad + q] = hv[d];
            b.ct_sl[c * npad + q] = (uint8_t)((sm >> e) & 1ull);
            ++c;
        }
    }
    b.ct_n[q] = c;
}

__global__ __launch_bounds__(256) void k_rb_copyback(Bufs b) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    b.dacc[q] = 0.0f;
    b.id[q] = b.alt_id[q];
    b.pos[q] = b.alt4[0][q];
    const double4 vh = b.alt4[1][q], wh = b.alt4[2][q];
    b.vh[q] = vh;
    b.wh[q] = wh;
    b.vf[q] = b.alt4[3][q];
    b.wf[q] = b.alt4[4][q];
    b.disp[q] = b.alt4[7][q];
    if (b.mixed) {
        const double4 f = b.alt4[5][q], t = b.alt4[6][q];
        ((float4*)b.F)[q] = make_float4((float)f.x, (float)f.y, (float)f.z, 0.0f);
        ((float4*)b.T)[q] = make_float4((float)t.x, (float)t.y, (float)t.z, 0.0f);
        b.vsh[q] = make_float4((float)vh.x, (float)vh.y, (float)vh.z, 0.0f);
        b.wsh[q] = make_float4((float)wh.x, (float)wh.y, (float)wh.z, 0.0f);
    } else {
        ((double4*)b.F)[q] = b.alt4[5][q];
        ((double4*)b.T)[q] = b.alt4[6][q];
    }
}

// Verlet list: every j with |r| <= (a_i + a_j) c_int + skin (c_int = 1 + xi_cut/2, or the
// repulsion's range factor when that is larger), sorted by
// partner id (so force sums do not depend on the cell layout), then the
// carried contact history is attached to its list entry.
__global__ __launch_bounds__(256) void k_rb_nlist(Bufs b, int q, int in_step) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t r = __builtin_amdgcn_readfirstlane(b.blk_rep[i / kTile]);
    const RepParams& P = b.reps[r];
    const uint32_t npad = b.npad, cap = b.cap;
    if (i - P.p_begin >= P.n) {
        b.ncnt[i] = 0u;
        b.cmask[i] = 0ull;
        b.smask[i] = 0ull;
        return;
    }
    const double4 pi = b.pos[i];
    const double s_base = b.dyn[r].s_slot[1 - q];
    const double s_le = in_step ? next_offset(P, s_base) : s_base;
    const double amax = P.rc_max / (2.0 * P.c_int);
    const double rli = (pi.w + amax) * P.c_int + P.skin;        // largest list radius of i
    const double margin = rli * (1.0 + 1e-12) + 1e-12 * P.L[0];
    const int cy = cell_coord(pi.y, P.cw[1], P.nc[1]);
    const int cz = cell_coord(pi.z, P.cw[2], P.nc[2]);
    uint32_t cnt = 0;
    const int oy0 = P.nc[1] == 1 ? 0 : -1, oy1 = P.nc[1] == 1 ? 0 : 1;
    const int oz0 = P.nc[2] == 1 ? 0 : -1, oz1 = P.nc[2] == 1 ? 0 : 1;
    for (int oz = oz0; oz <= oz1; ++oz) {
        const int zz = (cz + oz + P.nc[2]) % P.nc[2];
        for (int oy = oy0; oy <= oy1; ++oy) {
            int yy = cy + oy;
            double shift = 0.0;
            bool all_x = (P.nc[0] == 1) || (P.nc[1] == 1);
            if (yy < 0) { yy += P.nc[1]; shift = s_le; }          // j's image sits at y - Ly, x - s
            else if (yy >= P.nc[1]) { yy -= P.nc[1]; shift = -s_le; }
            const double xs = pi.x + shift;
            int xlo = (int)floor((xs - margin) / P.cw[0]);
            int xhi = (int)floor((xs + margin) / P.cw[0]);
            if (all_x || xhi - xlo + 1 >= P.nc[0]) { xlo = 0; xhi = P.nc[0] - 1; }
            for (int xc = xlo; xc <= xhi; ++xc) {
                const int xx = ((xc % P.nc[0]) + P.nc[0]) % P.nc[0];
                const uint32_t key = cell_key(P, xx, yy, zz);
                const uint32_t st = b.cell_start[key], en = st + b.cell_cnt[key];
                for (uint32_t j = st; j < en; ++j) {
                    if (j == i) continue;
                    const double4 pj = b.pos[j];
                    double dx, dy, dz;
                    min_image(P, s_le, pi, pj, dx, dy, dz);
                    const double d2 = (dx * dx + dy * dy) + dz * dz;
                    const double rl = (pi.w + pj.w) * P.c_int + P.skin;
                    if (d2 <= rl * rl) {
                        if (cnt < cap) b.nbr[cnt * npad + i] = j;
                        ++cnt;
                    }
                }
            }
        }
    }
    if (cnt > cap) {  // rare: the host regrows the lists to the largest count and builds them again
        atomicMax(&b.sys->list_need, cnt);
        cnt = cap;
    }
    // insertion sort of the entries by partner id
    for (uint32_t a = 1; a < cnt; ++a) {
        const uint32_t v = b.nbr[a * npad + i];
        const uint32_t idv = b.id[v];
        int c = (int)a - 1;
        while (c >= 0 && b.id[b.nbr[c * npad + i]] > idv) {
            b.nbr[(c + 1) * npad + i] = b.nbr[c * npad + i];
            --c;
        }
        b.nbr[(c + 1) * npad + i] = v;
    }
    b.ncnt[i] = cnt;
    // attach carried contact history
    uint64_t cm = 0ull, sm = 0ull;
    const uint32_t nct = b.ct_n[i];
    for (uint32_t c = 0; c < nct; ++c) {
        const uint32_t pid = b.ct_id[c * npad + i];
        for (uint32_t e = 0; e < cnt; ++e) {
            if (b.id[b.nbr[e * npad + i]] == pid) {
                double v[3];
                for (int d = 0; d < 3; ++d) v[d] = b.ct_s[(c * 3 + d) * npad + i];
                if (b.mixed) {
                    const float f[3] = {(float)v[0], (float)v[1], (float)v[2]};
                    store_spring<float>(b, e * npad + i, f);
                } else {
                    store_spring<double>(b, e * npad + i, v);
                }
                cm |= 1ull << e;
                if (b.ct_sl[c * npad + i]) sm |= 1ull << e;
                break;
            }
        }
    }
    b.cmask[i] = cm;
    b.smask[i] = sm;
}

// Mirror index of the half-pair evaluation: lo0 = first entry whose partner has
// the higher id (in pidx, whose mask it clears); for an entry with a lower-id
// partner j, the position of i in j's list (lists are symmetric: the range test
// is symmetric in i, j).
__global__ __launch_bounds__(256) void k_rb_mirror(Bufs b) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t r = __builtin_amdgcn_readfirstlane(b.blk_rep[i / kTile]);
    const RepParams& P = b.reps[r];
    const uint32_t npad = b.npad;
    if (i - P.p_begin >= P.n) {
        b.pidx[i] = PairIdx{0ull, 0u, 0u};
        return;
    }
    const uint32_t idi = b.id[i], cnt = b.ncnt[i];
    uint32_t e0 = cnt;
    for (uint32_t e = 0; e < cnt; ++e) {
        const uint32_t j = b.nbr[e * npad + i];
        if (b.id[j] > idi) {
            e0 = e;
            break;
        }
        const uint32_t cj = b.ncnt[j];
        uint32_t m = 0xFFu;
        for (uint32_t k = 0; k < cj; ++k)
            if (b.nbr[k * npad + j] == i) {
                m = k;
                break;
            }
        if (m == 0xFFu) {   // asymmetric lists: only truncated ones (then they are built again)
            if (b.sys->list_need == 0u) atomicOr(&b.dyn[r].health, H_NLIST);
            m = 0;
        }
        b.mir[e * npad + i] = (uint8_t)m;
    }
    b.pidx[i] = PairIdx{0ull, 0u, e0};
}

// after a build every list holds all pairs within range plus the full skin;
// q is the parity of the next force evaluation
__global__ void k_rb_reset(Bufs b, int q) {
    for (uint32_t r = threadIdx.x; r < b.nrep; r += blockDim.x) b.dyn[r].t_slot[1 - q] = 0.0;
    if (threadIdx.x == 0) {
        b.sys->halted = 0u;
        b.sys->expire[0] = 0u;
        b.sys->expire[1] = 0u;
        b.sys->rebuilds += 1;
    }
}

// clears the overflow record before a list build
__global__ void k_rb_need0(Bufs b) {
    if (threadIdx.x == 0) b.sys->list_need = 0u;
}

template <class R> struct Acc;
template <> struct Acc<double> {
    double v[3] = {0.0, 0.0, 0.0};
    __device__ __forceinline__ void add(int d, double x) { v[d] += x; }
    __device__ __forceinline__ double get(int d) const { return v[d]; }
};
// FP32 with Neumaier compensation
template <> struct Acc<float> {
    float s[3] = {0.f, 0.f, 0.f}, c[3] = {0.f, 0.f, 0.f};
    __device__ __forceinline__ void add(int d, float x) {
        const float t = s[d] + x;
        const float e = fabsf(s[d]) >= fabsf(x) ? (s[d] - t) + x : (x - t) + s[d];
        c[d] += e;
        s[d] = t;
    }
    __device__ __forceinline__ double get(int d) const { return (double)s[d] + (double)c[d]; }
};

// Precision policy: FP64 uses correctly rounded library operations; mixed
// precision uses the hardware FP32 log2, sqrt and reciprocal (about 1 ulp).
template <class R> __device__ __forceinline__ R rlog(R x);
template <> __device__ __forceinline__ double rlog<double>(double x) { return log(x); }
template <> __device__ __forceinline__ float rlog<float>(float x) {
    return 0.69314718055994531f * __builtin_amdgcn_logf(x);
}
template <class R> __device__ __forceinline__ void cross3r(const R* a, const R* b, R* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
template <class R> __device__ __forceinline__ R rexp(R x);
template <> __device__ __forceinline__ double rexp<double>(double x) { return exp(x); }
template <> __device__ __forceinline__ float rexp<float>(float x) {
    return __builtin_amdgcn_exp2f(1.4426950408889634f * x);
}
template <class R> __device__ __forceinline__ R rsqrt_(R x);
template <> __device__ __forceinline__ double rsqrt_<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float rsqrt_<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <class R> __device__ __forceinline__ R rrcp(R x);
// FP64: the hardware reciprocal refined by two Newton steps (within an ulp of 1/x; the
// springs, which the parity with the oracle needs to the bit, use correctly rounded
// divisions instead)
template <> __device__ __forceinline__ double rrcp<double>(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
template <> __device__ __forceinline__ float rrcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------------------
// Forces of a step with parity q: Sec. II.A-II.D pair terms, Sec. II.B-II.C
// one-body terms, kick 2.  The terms of particle i are a list of items: its
// interacting list entries in entry order (partner ids ascending), then a
// one-body force item (drag + noise) and a one-body torque item.  Every item
// draws one Philox block and three normals.  Pairs are evaluated once, in
// canonical orientation (r = x_i - x_j with i the lower id), so the pair
// forces are exactly antisymmetric; the stress of a pair is added once.  The
// force and torque on i are summed over its items in item order (FP64, or FP32
// with Neumaier compensation), so they do not depend on the launch shape.
// ---------------------------------------------------------------------------
constexpr uint32_t kItemForce = 64u;   // item code of the one-body force (list entries are < 64)
constexpr uint32_t kItemTorque = 65u;  // item code of the one-body torque

template <bool MIX> struct EvalCtx {
    using R = typename std::conditional<MIX, float, double>::type;
    double s_le, c1, invV;
    // the box: a pair loop that stores its results would otherwise read these from the
    // parameters again in every pass (eval_pair's BOXC; the FP64 occupancy form of the
    // half-pair kernel has no scalar registers to spare and reads them)
    double L[3], invL[3], gdLy;
    uint32_t k0, k1, ctr_lo, ctr_hi;
    R bamp, eta6pi, xi_min, kn, kt, mukn, dtR, repA, pieta;
    bool do_lub, do_br, do_ct, do_one, do_rep, do_rot;
};

// Step bookkeeping shared by the pair kernels.  eval_record: the writes of an
// evaluation that goes ahead, with its offset and step counter (first: this
// block is the first of its replica and records them, with the bound's time).
__device__ __forceinline__ void eval_record(const Bufs& b, int q, int advance, const RepParams& P, RepDyn& D,
                                            bool first, double s_le, uint64_t step, bool leader) {
    if (advance) {
        if (leader && threadIdx.x == 0) b.sys->expire[1 - q] = 0u;  // for the next step (one block of the launch)
        if (first && threadIdx.x == 0) {
            D.s_slot[q] = s_le;
            D.step_slot[q] = step;
            D.t_slot[q] = D.t_slot[1 - q] + P.dt;
            D.eval_seq += 1;
            D.eval_id[q] = D.eval_seq;
            D.nrec += 1;
            D.rec[q] = D.nrec;
        }
    } else if (first && threadIdx.x == 0) {
        D.eval_seq += 1;
        D.eval_id[q] = D.eval_seq;
        D.rec[q] = 0u;
    }
}

// values uniform over the wave (the evaluation's constants): readfirstlane keeps
// them in scalar registers whatever path they were loaded through
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ double uni(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = uni((uint32_t)u), hi = uni((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(lo | (hi << 32)));
}

// UNI: move the constants to scalar registers (pays where vector registers bind the
// occupancy; the kernels evaluating several items per lane run short of scalar ones)
template <bool MIX, bool UNI = false>
__device__ __forceinline__ void make_ctx(EvalCtx<MIX>& C, const RepParams& P, double s_le, uint64_t step) {
    using R = typename EvalCtx<MIX>::R;
    auto uni = [](auto v) { return UNI ? susp::uni(v) : v; };
    C.s_le = uni(s_le);
    for (int k = 0; k < 3; ++k) {
        C.L[k] = uni(P.L[k]);
        C.invL[k] = uni(P.invL[k]);
    }
    C.gdLy = uni(P.gdLy);
    C.c1 = uni(P.c1);
    C.invV = uni(P.invV);
    C.k0 = uni((uint32_t)P.seed);
    C.k1 = uni((uint32_t)(P.seed >> 32));
    C.ctr_lo = uni((uint32_t)step);
    C.ctr_hi = uni((uint32_t)(step >> 32) << 8);
    C.bamp = uni((R)P.bamp);
    C.eta6pi = uni((R)(6.0 * kPi * P.eta));
    C.xi_min = uni((R)P.xi_min);
    C.kn = uni((R)P.kn);
    C.kt = uni((R)P.kt);
    C.mukn = uni((R)(P.mu * P.kn));
    C.dtR = uni((R)P.dt);
    C.do_lub = !(P.flags & F_NO_LUB);
    C.do_br = !(P.flags & F_NO_PAIR_BROWN);
    C.do_ct = !(P.flags & F_NO_CONTACT);
    C.do_one = !(P.flags & F_NO_ONEBODY);
    C.repA = uni((R)P.rep_A);
    C.pieta = uni((R)kPi * (R)P.eta);
    C.do_rep = P.rep_A > 0.0;
    C.do_rot = (P.flags & F_LUB_ROT) != 0;
}

// interaction predicate of list entry j of particle i (exact FP64 test): gap xi <=
// xi_cut, or with the repulsion on, gap h <= 16 kappa (P.c_int = the larger range
// factor of the two)
__device__ __forceinline__ bool interacting(const RepParams& P, double s_le, const double4& pi, const double4& pj) {
    double dx, dy, dz;
    min_image(P, s_le, pi, pj, dx, dy, dz);
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    const double rc = (pi.w + pj.w) * P.c_int;
    return d2 <= rc * rc;
}

// One-body item of particle i from its three normals th: eq. (force_drag) +
// (force_brownian_drag) for e = kItemForce (into f), or eq. (torque_drag) +
// (torque_brownian_drag) for e = kItemTorque (into t).
template <bool MIX>
__device__ __forceinline__ void onebody_terms(const RepParams& P, const EvalCtx<MIX>& C, const double4& pi,
                                              uint32_t e, const typename EvalCtx<MIX>::R* vi,
                                              const typename EvalCtx<MIX>::R* wi, const typename EvalCtx<MIX>::R* th,
                                              typename EvalCtx<MIX>::R* f, typename EvalCtx<MIX>::R* t) {
    using R = typename EvalCtx<MIX>::R;
    const double a = pi.w;
    if (e == kItemForce) {
        const R zeta = (R)(6.0 * kPi * P.eta * a);
        const R sz = rsqrt_<R>(zeta);
        const R uinf[3] = {(R)(P.gd * (pi.y - 0.5 * P.L[1])), (R)0, (R)0};
#pragma unroll
        for (int d = 0; d < 3; ++d) f[d] = zeta * (uinf[d] - vi[d]) + C.bamp * sz * th[d];
    } else {
        const R zr = (R)(8.0 * kPi * P.eta * a * a * a);
        const R szr = rsqrt_<R>(zr);
        const R oinf[3] = {(R)0, (R)0, (R)(-0.5 * P.gd)};
#pragma unroll
        for (int d = 0; d < 3; ++d) t[d] = zr * (oinf[d] - wi[d]) + C.bamp * szr * th[d];
    }
}

// Partner data of a pair item loaded ahead of its evaluation (so that the
// loads of many items are in flight together).
template <class R> struct PairIn {
    uint32_t j, idj;
    double4 pj;
    R vj[3], wj[3], s[3];  // half-step velocities of j, stored spring of the entry
};

// One interacting pair (i, j), i the lower id (canonical orientation, r = x_i -
// x_j), from the partner data preloaded in `in`: the force f on i (j gets -f),
// the torque t on i, the spring update of list entry e of i, the contact and
// sliding bits, the largest overlap and the stress sums (addS).  tb_out: without
// ROT, n x (k_t s) of a contact (the torque per unit lever arm of both spheres);
// with ROT, the pair's torque on j.  EXT: the model extensions are compiled in
// (the short-ranged repulsion, which reaches beyond the lubrication cut-off, and
// the rotational lubrication couplings with the pairwise Brownian torques), each
// on when its parameter says.  BOXC: the box from the context (else from P).
// Returns false for a pair out of range (only when !BOXC; the half-pair kernel's
// cull tested the range with the same arithmetic otherwise).
template <bool MIX, bool EXT = false, bool BOXC = true, class AddS>
__device__ __forceinline__ bool eval_pair(const Bufs& b, const RepParams& P, const EvalCtx<MIX>& C, uint32_t i,
                                          uint32_t e, const double4& pi, uint32_t idi,
                                          const typename EvalCtx<MIX>::R* vi, const typename EvalCtx<MIX>::R* wi,
                                          bool had_contact, typename EvalCtx<MIX>::R* f,
                                          typename EvalCtx<MIX>::R* t, bool& contact, bool& slid, float& maxov,
                                          AddS addS, typename EvalCtx<MIX>::R* tb_out,
                                          const PairIn<typename EvalCtx<MIX>::R>& in) {
    using R = typename EvalCtx<MIX>::R;
    const uint32_t npad = b.npad;
    const R ai = (R)pi.w;
#pragma unroll
    for (int d = 0; d < 3; ++d) { f[d] = (R)0; t[d] = (R)0; }
    if (EXT) {  // with the couplings every pair has a torque record on j (zero for a repulsion-only pair)
#pragma unroll
        for (int d = 0; d < 3; ++d) tb_out[d] = (R)0;
    }
    contact = false;
    slid = false;
    // ---- geometry (FP64)
    const uint32_t idj = in.idj;
    const double4 pj = in.pj;
    double dx, dy, dz;
    const double* L = BOXC ? C.L : P.L;
    const double* invL = BOXC ? C.invL : P.invL;
    const int ky = min_image(L, invL, C.s_le, pi, pj, dx, dy, dz);
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    const double sa = pi.w + pj.w;
    const double rc = sa * C.c1;
    if (!BOXC && !(d2 <= rc * rc)) return false;
    // a pair the cull admitted for the repulsion alone (beyond the lubrication cut-off)
    const bool lubp = !(EXT && C.do_rep) || d2 <= rc * rc;
    const double dist = sqrt(d2);
    const double h = dist - sa;
    R n[3];
    const R inv = rrcp<R>((R)dist);
    n[0] = (R)dx * inv; n[1] = (R)dy * inv; n[2] = (R)dz * inv;
    const R aj = (R)pj.w;
    R XA = (R)0, YA = (R)0, lgv = (R)0;
    if (lubp) {
        const R xi = (R)(2.0 * h) * rrcp<R>((R)sa);
        const R xie = xi < C.xi_min ? C.xi_min : xi;
        // resistance scalars X^A_11, Y^A_11 (Sec. II.B) in the symmetric form
        const R pab = ai * aj, qab = ai * ai + aj * aj;
        const R sR = ai + aj;
        const R pre = C.eta6pi * rrcp<R>(sR * sR * sR);
        const R lg = -rlog<R>(xie);
        lgv = lg;
        XA = pre * ((R)2 * pab * pab * rrcp<R>(xie) + pab * (qab + (R)7 * pab) * (R)0.2 * lg);
        YA = pre * ((R)4 * pab * ((R)2 * qab + pab) * (R)(1.0 / 15.0) * lg);
    }
    // ---- one Philox block -> three normals
    R th[3] = {(R)0, (R)0, (R)0};
    if (C.do_br && lubp) {
        const uint4 w = philox10(C.ctr_lo, idi, idj, C.ctr_hi, C.k0, C.k1);  // stream 0
        normals3(w, th);
    }

    // ---- velocities; j's image moves with +k_y gammadot Ly
    R va[3], vb[3];
    const R shiftv = (R)((double)ky * (BOXC ? C.gdLy : P.gdLy));
#pragma unroll
    for (int d = 0; d < 3; ++d) { va[d] = vi[d]; vb[d] = in.vj[d]; }
    vb[0] = vb[0] + shiftv;

    R fl[3] = {(R)0, (R)0, (R)0}, fb[3] = {(R)0, (R)0, (R)0}, fc[3] = {(R)0, (R)0, (R)0};
    if (C.do_lub && lubp) {
        // eq. (force_lub): (X^A N + Y^A T)(U_j - U_i)
        R ur[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) ur[d] = vb[d] - va[d];
        const R un = (n[0] * ur[0] + n[1] * ur[1]) + n[2] * ur[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) fl[d] = XA * (un * n[d]) + YA * (ur[d] - un * n[d]);
    }
    if (C.do_br && lubp) {
        // eq. (force_brownian_lub): sqrt(2kT/dt) (sqrt(X^A) N + sqrt(Y^A) T) theta
        const R tn = (n[0] * th[0] + n[1] * th[1]) + n[2] * th[2];
        const R sx = rsqrt_<R>(XA), sy = rsqrt_<R>(YA);
#pragma unroll
        for (int d = 0; d < 3; ++d) fb[d] = C.bamp * (sx * (tn * n[d]) + sy * (th[d] - tn * n[d]));
    }
    const bool ROT = EXT && C.do_rot && lubp;
    R trot_a[3] = {(R)0, (R)0, (R)0}, trot_b[3] = {(R)0, (R)0, (R)0};
    if (ROT) {
        // Rotational couplings, eq. (force_lub), (torque_lub1), (torque_lub2), and pairwise
        // Brownian torques, eq. (torque_brownian_lub1), (torque_brownian_lub2).  The printed
        // signs hold for the unit vector from i to j, which is -n here; the scalars Y^B, Y^C
        // in the form symmetric in the radii.
        const R aa = ai, ab = aj;
        const R sR = aa + ab, i5s2 = (R)0.2 * rrcp<R>(sR * sR), isR = rrcp<R>(sR);
        const R pie = BOXC ? C.pieta : (R)kPi * (R)P.eta;
        const R YB11 = -(R)4 * pie * aa * aa * ab * ((R)4 * aa + ab) * i5s2 * lgv;
        const R YB21 = -(R)4 * pie * ab * ab * aa * ((R)4 * ab + aa) * i5s2 * lgv;
        const R YC11 = (R)3.2 * pie * aa * aa * aa * ab * isR * lgv;
        const R YC12 = (R)0.8 * pie * aa * aa * ab * ab * isR * lgv;  // = Y^C_21
        const R YC22 = (R)3.2 * pie * ab * ab * ab * aa * isR * lgv;
        const R nab[3] = {-n[0], -n[1], -n[2]};
        const R* wa = wi;
        const R* wb = in.wj;
        if (C.do_lub) {
            R ca[3], cb[3], urn[3], oa[3], ob[3];
            cross3r(wa, nab, ca);
            cross3r(wb, nab, cb);
#pragma unroll
            for (int d = 0; d < 3; ++d) fl[d] = fl[d] + (YB11 * ca[d] + YB21 * cb[d]);
            R ur[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) ur[d] = vb[d] - va[d];
            cross3r(ur, nab, urn);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                oa[d] = YC11 * wa[d] + YC12 * wb[d];
                ob[d] = YC12 * wa[d] + YC22 * wb[d];
            }
            const R oan = (n[0] * oa[0] + n[1] * oa[1]) + n[2] * oa[2];
            const R obn = (n[0] * ob[0] + n[1] * ob[1]) + n[2] * ob[2];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                trot_a[d] = YB11 * urn[d] - (oa[d] - oan * n[d]);
                trot_b[d] = YB21 * urn[d] - (ob[d] - obn * n[d]);
            }
        }
        if (C.do_br) {
            // the force's theta and a second vector chi (stream 1); a negative radicand is read as 0
            R chi[3], thn[3];
            normals3(philox10(C.ctr_lo, idi, idj, C.ctr_hi | 1u, C.k0, C.k1), chi);
            cross3r(th, nab, thn);
            const R cn = (n[0] * chi[0] + n[1] * chi[1]) + n[2] * chi[2];
            const R iya = rrcp<R>(YA);
            const R ra = YC11 - YB11 * YB11 * iya, rb = YC22 - YB21 * YB21 * iya;
            const R sa_ = ra > (R)0 ? rsqrt_<R>(ra) : (R)0, sb_ = rb > (R)0 ? rsqrt_<R>(rb) : (R)0;
            const R isya = rrcp<R>(rsqrt_<R>(YA));
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const R tchi = chi[d] - cn * n[d];
                trot_a[d] = trot_a[d] + C.bamp * (YB11 * isya * thn[d] + sa_ * tchi);
                trot_b[d] = trot_b[d] + C.bamp * (YB21 * isya * thn[d] + sb_ * tchi);
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) t[d] = trot_a[d];
#pragma unroll
        for (int d = 0; d < 3; ++d) tb_out[d] = trot_b[d];
    }
    if (h < 0.0 && C.do_ct) {
        // eq. (force_contact), (torque_contact); the spring s lives in canonical orientation
        const R aa = ai, ab = aj;
        const R delta = (R)(-h);
        if ((float)(-h) > maxov) maxov = (float)(-h);
        if (!MIX) {
            // the spring is updated with the correctly rounded normal (bit-reproducible history)
            const double dd = sqrt((dx * dx + dy * dy) + dz * dz);
            n[0] = (R)(dx / dd); n[1] = (R)(dy / dd); n[2] = (R)(dz / dd);
        }
        R s[3] = {(R)0, (R)0, (R)0};
        if (had_contact) {
#pragma unroll
            for (int d = 0; d < 3; ++d) s[d] = in.s[d];
        }
        R aw[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) aw[d] = aa * wi[d] + ab * in.wj[d];
        const R awn[3] = {aw[1] * n[2] - aw[2] * n[1], aw[2] * n[0] - aw[0] * n[2], aw[0] * n[1] - aw[1] * n[0]};
        R vc[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) vc[d] = (va[d] - vb[d]) - awn[d];
        const R vcn = (n[0] * vc[0] + n[1] * vc[1]) + n[2] * vc[2];
        R vt[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) vt[d] = vc[d] - vcn * n[d];
        const R sn = (n[0] * s[0] + n[1] * s[1]) + n[2] * s[2];
        R pr[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) pr[d] = s[d] - sn * n[d];
        const R ps = rsqrt_<R>((pr[0] * pr[0] + pr[1] * pr[1]) + pr[2] * pr[2]);
        if (ps > (R)0) {
            const R ss = rsqrt_<R>((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2]);
            const R fac = MIX ? ss * rrcp<R>(ps) : ss / ps;
#pragma unroll
            for (int d = 0; d < 3; ++d) s[d] = pr[d] * fac;
        } else {
#pragma unroll
            for (int d = 0; d < 3; ++d) s[d] = pr[d];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) s[d] = s[d] + C.dtR * vt[d];
        const R ftmax = C.mukn * delta;
        const R sl = rsqrt_<R>((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2]);
        if (C.kt * sl > ftmax) {
            const R fac = MIX ? ftmax * rrcp<R>(C.kt * sl) : ftmax / (C.kt * sl);
#pragma unroll
            for (int d = 0; d < 3; ++d) s[d] = s[d] * fac;
            slid = true;
        }
        store_spring_nt<R>(b, e * npad + i, s);
        contact = true;
        const R ks[3] = {C.kt * s[0], C.kt * s[1], C.kt * s[2]};
#pragma unroll
        for (int d = 0; d < 3; ++d) fc[d] = (C.kn * delta) * n[d] - ks[d];
        const R nks[3] = {n[1] * ks[2] - n[2] * ks[1], n[2] * ks[0] - n[0] * ks[2], n[0] * ks[1] - n[1] * ks[0]};
        if (ROT) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                t[d] = t[d] + ai * nks[d];
                tb_out[d] = tb_out[d] + aj * nks[d];
            }
        } else {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                t[d] = ai * nks[d];
                tb_out[d] = nks[d];
            }
        }
    }
    if (EXT && C.do_rep) {
        // short-ranged repulsion (A / kappa) exp(-h / kappa) n, kappa = 0.01 (a_i + a_j) (Sec. IV.F),
        // an interparticle force like contact: it joins fc (and the contact stress)
        const R kappa = (R)(0.01 * (pi.w + pj.w));
        const R fr = C.repA * rrcp<R>(kappa) * rexp<R>(-(R)h * rrcp<R>(kappa));
#pragma unroll
        for (int d = 0; d < 3; ++d) fc[d] = fc[d] + fr * n[d];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) f[d] = fl[d] + fb[d] + fc[d];
    // Sec. II.A, II.B, II.D: Sigma^X_ab -= F^X_a r_b / V, FP64
    const double rr[3] = {dx * C.invV, dy * C.invV, dz * C.invV};
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int be = 0; be < 3; ++be) {
            addS(3 * al + be, -(double)fc[al] * rr[be]);
            addS(9 + 3 * al + be, -(double)fl[al] * rr[be]);
            addS(18 + 3 * al + be, -(double)fb[al] * rr[be]);
        }
    return true;
}

// i-side velocities as used by the pair arithmetic
template <bool MIX>
__device__ __forceinline__ void load_vw(const Bufs& b, uint32_t i, typename EvalCtx<MIX>::R* vi,
                                        typename EvalCtx<MIX>::R* wi) {
    using R = typename EvalCtx<MIX>::R;
    if (MIX) {
        const float4 v4 = b.vsh[i], w4 = b.wsh[i];
        vi[0] = v4.x; vi[1] = v4.y; vi[2] = v4.z;
        wi[0] = w4.x; wi[1] = w4.y; wi[2] = w4.z;
    } else {
        const double4 v4 = b.vh[i], w4 = b.wh[i];
        vi[0] = (R)v4.x; vi[1] = (R)v4.y; vi[2] = (R)v4.z;
        wi[0] = (R)w4.x; wi[1] = (R)w4.y; wi[2] = (R)w4.z;
    }
}

__device__ __forceinline__ bool nonfinite(const double* Ft, const double* Tt) {
    return !(isfinite(Ft[0]) && isfinite(Ft[1]) && isfinite(Ft[2]) && isfinite(Tt[0]) && isfinite(Tt[1]) &&
             isfinite(Tt[2]));
}
template <bool MIX>
__device__ __forceinline__ void store_ft(const Bufs& b, uint32_t i, const double* Ft, const double* Tt) {
    if (MIX) {
        ((float4*)b.F)[i] = make_float4((float)Ft[0], (float)Ft[1], (float)Ft[2], 0.0f);
        ((float4*)b.T)[i] = make_float4((float)Tt[0], (float)Tt[1], (float)Tt[2], 0.0f);
    } else {
        ((double4*)b.F)[i] = make_double4(Ft[0], Ft[1], Ft[2], 0.0);
        ((double4*)b.T)[i] = make_double4(Tt[0], Tt[1], Tt[2], 0.0);
    }
}
// ---------------------------------------------------------------------------
// Half-pair evaluation: every interacting pair is evaluated once, by its
// lower-id particle.  k_half: a wave owns NP = 64 / LN particles; LN lanes
// per particle test the entries whose partner has the higher id (a suffix of
// the id-sorted list), the wave packs the interacting ones into a queue and
// evaluates them 64 at a time, writing the pair force on the lower-id
// particle and, for a contact, n x (k_t s), in queue order.  More lanes per
// particle suit systems too small to fill the GPU with one.  k_gather: each
// lane sums its particle's pair terms in entry order (reading a lower-id
// partner's result through the mirror index, negated), then the one-body
// force and torque, then applies kick 2.  The sums run in item order whatever
// the lanes per particle, the queue rounds or the particle layout, so forces,
// torques and springs do not depend on them.
// ---------------------------------------------------------------------------

// OCC (FP64 without the model extensions): the form for occupancy -- the queue is
// processed in rounds of kQCap items and 13 of the 27 stress sums live in LDS, so
// that the kernel fits 3 waves per SIMD; it pays on systems that fill the GPU many
// times over, while small ones (one round of waves) want the shortest wave.
template <bool MIX, int LN, bool EXT, bool OCC = false>
__global__ __launch_bounds__(256, (MIX || OCC) ? 3 : 2) void k_half(Bufs b, int q, int advance, uint32_t only_rep) {
    using R = typename std::conditional<MIX, float, double>::type;
    using V3 = typename PairRec<R>::T;
    constexpr int NP = 64 / LN;  // particles per wave
    // the first blocks (27 * nrep, padded to a multiple of 8 so that the XCD order of
    // the pair blocks is kept) reduce the stress of the previous evaluation (its
    // partials have the other parity): dispatched first, they run beside the pair blocks
    const uint32_t nfin = (27u * b.nrep + 7u) & ~7u, npair_blk = gridDim.x - nfin;
    if (blockIdx.x < nfin) {
        if (blockIdx.x >= 27u * b.nrep || b.sys->halted) return;
        finalize_unit(b, blockIdx.x / 27u, (int)(blockIdx.x % 27u), 1 - q);
        return;
    }
    const int w = threadIdx.x >> 6, p = threadIdx.x & 63;
    const uint32_t tile = xcd_tile(blockIdx.x - nfin, npair_blk);  // a block: 4 NP particles, inside one kTile
    const uint32_t base = (tile * 4 + w) * NP;                // first particle of this wave
    const uint32_t l = p / LN, sub = p % LN;
    const uint32_t i = base + l;
    const uint32_t npad = b.npad;
    // The cull reads only list and position data, which stay in bounds whatever the
    // step's state, and padding slots have empty lists: it runs before any exit test,
    // so that its loads are issued at once, beside those of the replica's parameters
    // and the step's bookkeeping, rather than after a chain of dependent checks.
    // (Loads complete in issue order: the ones needed first are issued first.)
    // (r is the same for the whole wave: readfirstlane keeps it, and what derives from
    // the replica's parameters, such as the noise keys, in scalar registers)
    const uint32_t r = __builtin_amdgcn_readfirstlane(b.blk_rep[base / kTile]);
    const uint32_t halted = b.sys->halted, expired = b.sys->expire[q] & (advance ? ~0u : 0u);
    const uint32_t cnt = min(b.ncnt[i], b.cap), e_lo = b.pidx[i].lo0;
    const double4 pi = b.pos[i];
    const uint64_t cm_i = b.cmask[i];
    // the first group of partners as well in FP64 (in mixed precision, where the
    // evaluation is shorter, the early group measured slower)
    constexpr uint32_t G0 = MIX ? 0u : 4u;
    uint32_t jj0[4];
    double4 pj0[4];
    if constexpr (G0 > 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // slots past the count hold stale indices: loaded, not used
            const uint32_t e = e_lo + sub + u * LN;
            const uint32_t j = b.nbr[min(e, b.cap - 1u) * npad + i];
            jj0[u] = e < cnt ? j : i;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) pj0[u] = b.pos[jj0[u]];
    }
    const RepParams& P = b.reps[r];
    RepDyn& D = b.dyn[r];
    // offset and step counter of this evaluation (its bookkeeping writes follow the
    // exit tests)
    const double s_le = advance ? next_offset(P, D.s_slot[1 - q]) : D.s_slot[q];
    const uint64_t step = advance ? D.step_slot[1 - q] + 1 : D.step_slot[q];

    // exit tests and the step's bookkeeping, after the cull
    auto go = [&]() -> bool {
        if (halted) return false;
        if (only_rep != 0xFFFFFFFFu && r != only_rep) return false;
        if (expired) {
            if (blockIdx.x == nfin && threadIdx.x == 0) b.sys->halted = 1u;
            return false;
        }
        eval_record(b, q, advance, P, D, tile == P.p_begin / (4 * NP), s_le, step, blockIdx.x == nfin);
        return true;
    };

    // ---- cull: interacting entries with a higher-id partner (LN lanes per particle).
    // Without OCC the partner index of the particle's first kJC higher-id entries stays
    // in LDS, so that the evaluation of those pairs needs no second read of the list
    // (with OCC the LDS goes to the queue instead: the cache measured slower there).
    constexpr uint32_t kJC = OCC ? 0u : 8u;
    __shared__ uint32_t jcache[4][NP][kJC > 0 ? kJC : 1];
    __shared__ uint8_t elo_s[4][NP];
    if (kJC > 0 && sub == 0) elo_s[w][l] = (uint8_t)e_lo;
    uint64_t im = 0ull;
    if constexpr (G0 > 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t e = e_lo + sub + u * LN;
            if (kJC > 0 && e < cnt && e - e_lo < kJC) jcache[w][l][e - e_lo] = jj0[u];
            if (e < cnt && interacting(P, s_le, pi, pj0[u])) im |= 1ull << e;
        }
    }
    for (uint32_t c0 = e_lo + sub + G0 * LN; c0 < cnt; c0 += 4 * LN) {
        uint32_t jj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t e = c0 + u * LN;
            jj[u] = e < cnt ? b.nbr[e * npad + i] : i;
        }
        double4 pj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pj[u] = b.pos[jj[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t e = c0 + u * LN;
            if (kJC > 0 && e < cnt && e - e_lo < kJC) jcache[w][l][e - e_lo] = jj[u];
            if (e < cnt && interacting(P, s_le, pi, pj[u])) im |= 1ull << e;
        }
    }

    // (the constants are read before the bookkeeping's stores: after them the
    // compiler would read them again from memory)
    EvalCtx<MIX> C;
    make_ctx<MIX, true>(C, P, s_le, step);
    if (!go()) return;

    // The queue holds up to qc items of a wave at a time: all of them (NP * 64), or with
    // OCC b.qcap <= 2048 (a wave's interacting pairs seldom exceed a few hundred; more
    // are evaluated in further rounds).
    constexpr uint32_t kQCap = OCC ? 2048u : (uint32_t)NP * 64u;
    const uint32_t qc = OCC ? min(b.qcap, kQCap) : kQCap;
    __shared__ uint16_t queue[4][kQCap];   // (particle slot << 6) | entry
    __shared__ unsigned long long cmo[4][NP], cmq[4][NP], smq[4][NP];
    const bool valid = i - P.p_begin < P.n;
    if (valid && sub == 0) cmo[w][l] = cm_i;
    if (LN >= 2) im |= dpp_u64<0xB1>(im);
    if (LN >= 4) im |= dpp_u64<0x4E>(im);
    if (sub == 0) {
        cmq[w][l] = 0ull;
        smq[w][l] = 0ull;
    }
    // exclusive prefix of the per-particle counts across the wave
    const uint32_t cnt_i = sub == 0 ? (uint32_t)__popcll(im) : 0u;
    uint32_t incl = cnt_i;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off);
        if (p >= off) incl += y;
    }
    const uint32_t total = __shfl(incl, 63);
    const uint32_t qk0 = incl - cnt_i;  // the particle's first position in the wave's queue order
    if (sub == 0 && valid) {
        b.pidx[i] = PairIdx{im, qk0, e_lo};
    }
    // results of this wave's pairs: a contiguous run in queue order
    V3* const pf = (V3*)b.pf + (size_t)base * b.cap;
    V3* const pt = (V3*)b.pt + (size_t)base * b.cap;
    V3* const pt2 = (V3*)b.pt2 + (size_t)base * b.cap;

    // ---- evaluate the queue, one pair per lane
    // stress sums: the first NR components in registers, the others in per-lane LDS
    // slots (one writer each); the same additions in the same order either way
    constexpr int NR = OCC && !MIX ? 14 : 27, NL = 27 - NR;
    __shared__ double sacc[NL > 0 ? NL : 1][NL > 0 ? 256 : 1];
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;
#pragma unroll
    for (int c = 0; c < NL; ++c) sacc[c][threadIdx.x] = 0.0;
    auto addS = [&](int c, double v) {
        if (c < NR) acc[c < NR ? c : 0] += v;
        else sacc[c < NR ? 0 : c - NR][threadIdx.x] += v;
    };
    float maxov = 0.0f;
    // one pair: item k of the wave's queue order, code (particle slot << 6) | entry
    auto do_pair = [&](uint32_t k, uint32_t code) {
        const uint32_t l = code >> 6, e = code & 63u;
        const uint32_t ii = base + l;
        const bool had = (cmo[w][l] >> e) & 1ull;
        // own data and the list entry, then the partner's data and the spring, each
        // group of loads in flight together
        const double4 pi = b.pos[ii];
        const uint32_t idi = b.id[ii];
        R vi[3], wi[3];
        load_vw<MIX>(b, ii, vi, wi);
        PairIn<R> in;
        if constexpr (kJC > 0) {
            const uint32_t ec = e - elo_s[w][l];   // entries past the cache are read from the list again
            in.j = ec < kJC ? jcache[w][l][ec] : b.nbr[e * npad + ii];
        } else {
            in.j = b.nbr[e * npad + ii];
        }
        in.pj = b.pos[in.j];
        in.idj = b.id[in.j];
        load_vw<MIX>(b, in.j, in.vj, in.wj);
        if (had) load_spring_nt<R>(b, e * npad + ii, in.s);
        else in.s[0] = in.s[1] = in.s[2] = (R)0;
        R f[3], t[3], tb[3];  // tb: written by eval_pair where it is used (contact, or the couplings)
        bool contact, slid;
        eval_pair<MIX, EXT, MIX || !OCC>(b, P, C, ii, e, pi, idi, vi, wi, had, f, t, contact, slid, maxov, addS, tb,
                                         in);
        pf[k] = PairRec<R>::make(f[0], f[1], f[2]);
        if (EXT && C.do_rot) {  // torques on the lower- and the higher-id particle
            pt[k] = PairRec<R>::make(t[0], t[1], t[2]);
            pt2[k] = PairRec<R>::make(tb[0], tb[1], tb[2]);
        } else if (contact) {  // n x (k_t s): each side scales it by its radius
            pt[k] = PairRec<R>::make(tb[0], tb[1], tb[2]);
        }
        if (contact) {
            atomicOr(&cmq[w][l], 1ull << e);
            if (slid) atomicOr(&smq[w][l], 1ull << e);
        }
    };
    auto fill = [&](uint32_t r0) {  // the items of positions [r0, r0 + qc) of the queue order
        if (sub == 0) {
            uint32_t k = qk0;
            for (uint64_t m = im; m; m &= m - 1ull, ++k)
                if (k - r0 < qc) queue[w][k - r0] = (uint16_t)((l << 6) | __builtin_ctzll(m));
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };
    if constexpr (OCC) {
        for (uint32_t r0 = 0; r0 < total; r0 += qc) {
            fill(r0);
            const uint32_t nq = min(total - r0, qc);
            for (uint32_t kq = p; kq < nq; kq += 64) do_pair(r0 + kq, queue[w][kq]);
            __builtin_amdgcn_wave_barrier();  // the queue is refilled by the next round
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
    } else {  // one round holds every item
        if (sub == 0) {
            uint32_t k = qk0;
            for (uint64_t m = im; m; m &= m - 1ull) queue[w][k++] = (uint16_t)((l << 6) | __builtin_ctzll(m));
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (uint32_t k = p; k < total; k += 64) do_pair(k, queue[w][k]);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (valid && sub == 0) {
        b.cmask[i] = cmq[w][l];
        __builtin_nontemporal_store((unsigned long long)smq[w][l], (unsigned long long*)&b.smask[i]);   // read at list builds
    }

    // block partial of the stress (fixed-order sum over the block's lanes: DPP rows,
    // then LDS) and the block's largest overlap, behind one barrier
    __shared__ double rows[16][27];
    __shared__ float mrows[16];
    maxov = fmaxf(maxov, dpp_f32<0x111>(maxov));
    maxov = fmaxf(maxov, dpp_f32<0x112>(maxov));
    maxov = fmaxf(maxov, dpp_f32<0x114>(maxov));
    maxov = fmaxf(maxov, dpp_f32<0x118>(maxov));
    if ((p & 15) == 15) mrows[threadIdx.x >> 4] = maxov;
#pragma unroll
    for (int c = 0; c < 27; ++c) {
        const double v = row_sum_f64(c < NR ? acc[c < NR ? c : 0] : sacc[c < NR ? 0 : c - NR][threadIdx.x]);
        if ((p & 15) == 15) rows[threadIdx.x >> 4][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 27) {
        const int c = threadIdx.x;
        double tsum = 0.0;
        for (int k = 0; k < 16; ++k) tsum += rows[k][c];
        b.partial[((size_t)q * 27 + c) * b.nblk_max + tile] = tsum;
    } else if (threadIdx.x == 32) {
        float m = mrows[0];
        for (int k = 1; k < 16; ++k) m = fmaxf(m, mrows[k]);
        b.ovpart[(size_t)q * b.nblk_max + tile] = m;
    }
}

template <bool MIX, bool ROT>
__device__ __forceinline__ void gather_particle(const Bufs& b, const RepParams& P, const RepDyn& D, int q, int kick,
                                                int fuse, uint32_t i, float& dblk, bool& expire, bool& bad,
                                                uint32_t halted);

// fuse: also take kick 1 and the drift of the next step (parity 1 - q) from the
// new forces, as the integrate launch of that step would.  The halted test follows
// the particle's own loads (all in bounds whatever the step's state), so that they
// are in flight beside the flag's.
template <bool MIX, bool ROT>
__global__ __launch_bounds__(256) void k_gather(Bufs b, int q, int kick, int fuse, uint32_t only_rep) {
    const uint32_t halted = b.sys->halted;
    const uint32_t tile = xcd_tile_rev(blockIdx.x, gridDim.x);
    const uint32_t i = tile * 256 + threadIdx.x;
    const uint32_t r = __builtin_amdgcn_readfirstlane(b.blk_rep[tile]);
    if (only_rep != 0xFFFFFFFFu && r != only_rep) return;
    const RepParams& P = b.reps[r];
    RepDyn& D = b.dyn[r];
    float dblk = 0.0f;
    bool expire = false, bad = false;
    if (i - P.p_begin < P.n) gather_particle<MIX, ROT>(b, P, D, q, kick, fuse, i, dblk, expire, bad, halted);
    if (halted) return;
    if (bad) atomicOr(&D.health, H_NAN);
    if (fuse) {
        if (expire) atomicOr(&b.sys->expire[1 - q], 1u);
        block_max_store(dblk, &b.dpart[(size_t)(1 - q) * (b.npad / kTile) + tile]);
    }
}

template <bool MIX, bool ROT>
__device__ __forceinline__ void gather_particle(const Bufs& b, const RepParams& P, const RepDyn& D, int q, int kick,
                                                int fuse, uint32_t i, float& dblk, bool& expire, bool& bad,
                                                uint32_t halted) {
    using R = typename std::conditional<MIX, float, double>::type;
    using V3 = typename PairRec<R>::T;
    EvalCtx<MIX> C;
    make_ctx<MIX, true>(C, P, D.s_slot[q], D.step_slot[q]);
    const DriftPar dp = drift_par(P, D, 1 - q);  // the next step's (fused steps)
    const uint32_t npad = b.npad, cap = b.cap;
    const double4 pi = b.pos[i];
    const uint32_t idi = b.id[i];
    const R ai = (R)pi.w;
    // the half-step velocities for the one-body terms and the kicks (in mixed precision the
    // FP32 copies are these values rounded, so they are not read again)
    const double4 vh = MIX ? ld_nt(&b.vh[i]) : b.vh[i], wh = MIX ? ld_nt(&b.wh[i]) : b.wh[i];
    const R vi[3] = {(R)vh.x, (R)vh.y, (R)vh.z}, wi[3] = {(R)wh.x, (R)wh.y, (R)wh.z};
    Acc<R> F, T;
    const PairIdx pq = b.pidx[i];
    const uint32_t e0 = pq.lo0;
    const uint64_t im = pq.im, cm = b.cmask[i];
    const uint32_t wmask = ~(64u / (uint32_t)b.lanes - 1u);
    const size_t kw = (size_t)(i & wmask) * cap, k0 = kw + pq.qoff;
    if (halted) return;
    // Pair k of the wave owning particle p sits at (p & ~(NP - 1)) * cap + k, NP = 64 /
    // lanes.  First the entries [0, e0), whose partner j has the lower id: entry m of j's
    // list holds the pair, and j's records run in the order of its interacting entries.
    // Groups of GB entries, each stage's loads issued together.  No load sits behind a
    // branch (a lane without an item reads its wave's first record instead), nor does a sum:
    // such a lane adds +0, which leaves a sum that starts at +0 unchanged.
    constexpr uint32_t GB = 4;
    for (uint32_t c0 = 0; c0 < e0; c0 += GB) {
        uint32_t jj[GB], mm[GB], qj[GB];
        uint64_t imj[GB], cmj[GB];
#pragma unroll
        for (uint32_t u = 0; u < GB; ++u) {
            const uint32_t e = min(c0 + u, e0 - 1u);
            jj[u] = b.nbr[e * npad + i];
            mm[u] = b.mir[e * npad + i];
        }
#pragma unroll
        for (uint32_t u = 0; u < GB; ++u) {
            const PairIdx pj = b.pidx[jj[u]];
            imj[u] = pj.im;
            qj[u] = pj.qoff;
            cmj[u] = ROT ? 0ull : b.cmask[jj[u]];
        }
        V3 fv[GB], tv[GB];
        bool use[GB], ct[GB];
#pragma unroll
        for (uint32_t u = 0; u < GB; ++u) {
            use[u] = c0 + u < e0 && ((imj[u] >> mm[u]) & 1ull);
            ct[u] = use[u] && (ROT || ((cmj[u] >> mm[u]) & 1ull));
            const size_t slot =
                (size_t)(jj[u] & wmask) * cap + qj[u] + (uint32_t)__popcll(imj[u] & ((1ull << mm[u]) - 1ull));
            fv[u] = ((const V3*)b.pf)[use[u] ? slot : kw];
            // with ROT the record of the torque on the higher-id particle
            tv[u] = ((const V3*)(ROT ? b.pt2 : b.pt))[ct[u] ? slot : kw];
        }
#pragma unroll
        for (uint32_t u = 0; u < GB; ++u) {
            F.add(0, use[u] ? (R)-1 * fv[u].x : (R)0);
            F.add(1, use[u] ? (R)-1 * fv[u].y : (R)0);
            F.add(2, use[u] ? (R)-1 * fv[u].z : (R)0);
            // without ROT the record is n x (k_t s): each side scales it by its radius
            T.add(0, ct[u] ? (ROT ? tv[u].x : ai * tv[u].x) : (R)0);
            T.add(1, ct[u] ? (ROT ? tv[u].y : ai * tv[u].y) : (R)0);
            T.add(2, ct[u] ? (ROT ? tv[u].z : ai * tv[u].z) : (R)0);
        }
    }
    // then the particle's own pairs (entries from e0 on that interact): a contiguous run
    // from k0, in entry order
    const uint32_t nown = (uint32_t)__popcll(im);
    uint64_t rest = im;
    for (uint32_t c0 = 0; c0 < nown; c0 += GB) {
        V3 fv[GB], tv[GB];
        bool use[GB], ct[GB];
#pragma unroll
        for (uint32_t u = 0; u < GB; ++u) {
            use[u] = c0 + u < nown;
            const uint32_t e = rest ? (uint32_t)__builtin_ctzll(rest) : 0u;
            rest &= rest - 1ull;
            ct[u] = use[u] && (ROT || ((cm >> e) & 1ull));
            fv[u] = ((const V3*)b.pf)[use[u] ? k0 + c0 + u : kw];
            tv[u] = ((const V3*)b.pt)[ct[u] ? k0 + c0 + u : kw];
        }
#pragma unroll
        for (uint32_t u = 0; u < GB; ++u) {
            F.add(0, use[u] ? fv[u].x : (R)0);
            F.add(1, use[u] ? fv[u].y : (R)0);
            F.add(2, use[u] ? fv[u].z : (R)0);
            T.add(0, ct[u] ? (ROT ? tv[u].x : ai * tv[u].x) : (R)0);
            T.add(1, ct[u] ? (ROT ? tv[u].y : ai * tv[u].y) : (R)0);
            T.add(2, ct[u] ? (ROT ? tv[u].z : ai * tv[u].z) : (R)0);
        }
    }
    // what the drift reads, issued here (before any store of the launch) so that the
    // one-body terms hide the wait
    double4 da = make_double4(0.0, 0.0, 0.0, 0.0);
    double dacc = 0.0;
    if (fuse) {
        if (dp.flags & F_TRACK_DISP) da = b.disp[i];
        dacc = __builtin_nontemporal_load(&b.dacc[i]);   // read once per step
    }
    if (C.do_one) {
#pragma unroll
        for (uint32_t e = kItemForce; e <= kItemTorque; ++e) {
            R th[3], f[3], t[3];
            const uint4 u = philox10(C.ctr_lo, idi, 0xFFFFFFFFu, C.ctr_hi | (e == kItemForce ? 2u : 3u), C.k0, C.k1);
            normals3(u, th);
            onebody_terms<MIX>(P, C, pi, e, vi, wi, th, f, t);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (e == kItemForce) F.add(d, f[d]);
                else T.add(d, t[d]);
            }
        }
    }
    double Ft[3], Tt[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) { Ft[d] = F.get(d); Tt[d] = T.get(d); }
    bad = nonfinite(Ft, Tt);
    // kick 2; a fused step keeps the full-step values in registers: only the last step
    // of a launch sequence (never fused) leaves them in memory for the state readers
    double4 vf = vh, wf = wh;
    if (kick) half_kick(pi.w, dp.rho, dp.half_dt, Ft, Tt, vf, wf);
    if (!fuse) {
        store_ft<MIX>(b, i, Ft, Tt);
        b.vf[i] = vf;
        b.wf[i] = wf;
    } else {
        if (MIX) {  // the next kick uses the force as stored
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                Ft[d] = (double)(float)Ft[d];
                Tt[d] = (double)(float)Tt[d];
            }
        }
        integrate_particle<MIX>(b, dp, i, pi, vf, wf, Ft, Tt, da, dacc, dblk, expire);
    }
}

// Mean-square non-affine displacement sums of one replica (the MSD of
// Sec. III.B): part[block * 3 + d] = fixed-order block sum of disp_d^2.
__global__ __launch_bounds__(256) void k_msd(Bufs b, uint32_t rep, double* part) {
    const RepParams& P = b.reps[rep];
    const uint32_t i = P.p_begin + blockIdx.x * 256 + threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    if (i - P.p_begin < P.n) {
        const double4 d = b.disp[i];
        acc[0] = d.x * d.x; acc[1] = d.y * d.y; acc[2] = d.z * d.z;
    }
    __shared__ double rows[16][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double v = row_sum_f64(acc[c]);
        if ((threadIdx.x & 15) == 15) rows[threadIdx.x >> 4][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += rows[k][threadIdx.x];
        part[blockIdx.x * 3 + threadIdx.x] = t;
    }
}

// Kinetic temperatures of one replica from its full-step velocities: per block the
// fixed-order sums of m |v - U^inf(x)|^2 and I |w - Omega^inf|^2 (peculiar
// translational and rotational motion; m = 4/3 pi rho a^3, I = 2/5 m a^2).
__global__ __launch_bounds__(256) void k_kinetic(Bufs b, uint32_t rep, double* part) {
    const RepParams& P = b.reps[rep];
    const uint32_t i = P.p_begin + blockIdx.x * 256 + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (i - P.p_begin < P.n) {
        const double4 x = b.pos[i], v = b.vf[i], w = b.wf[i];
        const double m = (4.0 / 3.0) * kPi * P.rho * x.w * x.w * x.w;
        const double I = 0.4 * m * x.w * x.w;
        const double ux = v.x - P.gd * (x.y - 0.5 * P.L[1]), wz = w.z + 0.5 * P.gd;
        acc[0] = m * ((ux * ux + v.y * v.y) + v.z * v.z);
        acc[1] = I * ((w.x * w.x + w.y * w.y) + wz * wz);
    }
    __shared__ double rows[16][2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double v = row_sum_f64(acc[c]);
        if ((threadIdx.x & 15) == 15) rows[threadIdx.x >> 4][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += rows[k][threadIdx.x];
        part[blockIdx.x * 2 + threadIdx.x] = t;
    }
}

void launch_kinetic(const Bufs& b, hipStream_t st, uint32_t rep, uint32_t nblk, double* part) {
    hipLaunchKernelGGL(k_kinetic, dim3(nblk), dim3(256), 0, st, b, rep, part);
}

void launch_msd(const Bufs& b, hipStream_t st, uint32_t rep, uint32_t nblk, double* part) {
    hipLaunchKernelGGL(k_msd, dim3(nblk), dim3(256), 0, st, b, rep, part);
}

// Pair histograms of one replica at parity p from its own cell pass (any range
// below half the box, independent of the lists): every particle scans the cells
// within `reach` of it -- across the sheared y boundary the x range is shifted by
// the Lees-Edwards offset -- and takes each partner with a higher id once, over
// the minimum image r = x_i - x_j.
//   mode 0 (g(r), Sec. III.A): |r| < r_max into nbins bins of width r_max / nbins;
//   mode 1 (slice of g through the flow-gradient plane, Sec. IV.D): pairs with
//     |r_z| < slab / 2 and |r_x|, |r_y| < r_max, binned by (r_x, r_y) on an
//     nbins x nbins grid over [-r_max, r_max)^2, each pair at r and at -r;
//     counts[ix * nbins + iy].
// Integer counts, so the order of the atomic increments does not matter.
__device__ __forceinline__ void rdf_bin(double dx, double dy, double dz, int mode, double r_max, double slab,
                                        uint32_t nbins, unsigned long long* counts) {
    if (mode == 0) {
        const double r = sqrt((dx * dx + dy * dy) + dz * dz);
        if (!(r < r_max)) return;
        uint32_t k = (uint32_t)(r / r_max * (double)nbins);
        if (k >= nbins) k = nbins - 1;
        atomicAdd(&counts[k], 1ull);
    } else {
        if (!(fabs(dz) < 0.5 * slab) || !(fabs(dx) < r_max) || !(fabs(dy) < r_max)) return;
        const double w = 2.0 * r_max;
        for (int sgn = 0; sgn < 2; ++sgn) {
            const double ux = sgn ? -dx : dx, uy = sgn ? -dy : dy;
            uint32_t ix = (uint32_t)((ux + r_max) / w * (double)nbins), iy = (uint32_t)((uy + r_max) / w * (double)nbins);
            if (ix >= nbins) ix = nbins - 1;
            if (iy >= nbins) iy = nbins - 1;
            atomicAdd(&counts[(size_t)ix * nbins + iy], 1ull);
        }
    }
}

__global__ __launch_bounds__(256) void k_rdf(Bufs b, uint32_t rep, int p, int mode, double r_max, double slab,
                                             double reach, uint32_t nbins, unsigned long long* counts) {
    const RepParams& P = b.reps[rep];
    const uint32_t i = P.p_begin + blockIdx.x * 256 + threadIdx.x;
    if (i - P.p_begin >= P.n) return;
    const double4 pi = b.pos[i];
    const uint32_t idi = b.id[i];
    const double s_le = b.dyn[rep].s_slot[p];
    const double margin = reach * (1.0 + 1e-12) + 1e-12 * P.L[0];
    const int cy = cell_coord(pi.y, P.cw[1], P.nc[1]);
    const int cz = cell_coord(pi.z, P.cw[2], P.nc[2]);
    int ly = (int)ceil(margin / P.cw[1]), lz = (int)ceil(margin / P.cw[2]);
    // rows (y) or layers (z) scanned all at once when the layers would wrap onto themselves
    const bool all_y = 2 * ly + 1 >= P.nc[1], all_z = 2 * lz + 1 >= P.nc[2];
    const int oy0 = all_y ? 0 : -ly, oy1 = all_y ? P.nc[1] - 1 : ly;
    const int oz0 = all_z ? 0 : -lz, oz1 = all_z ? P.nc[2] - 1 : lz;
    for (int oz = oz0; oz <= oz1; ++oz) {
        const int zz = all_z ? oz : ((cz + oz) % P.nc[2] + P.nc[2]) % P.nc[2];
        for (int oy = oy0; oy <= oy1; ++oy) {
            int yy = all_y ? oy : cy + oy;
            double shift = 0.0;
            if (!all_y) {
                if (yy < 0) { yy += P.nc[1]; shift = s_le; }             // j's image sits at y - Ly, x - s
                else if (yy >= P.nc[1]) { yy -= P.nc[1]; shift = -s_le; }
            }
            const double xs = pi.x + shift;
            int xlo = (int)floor((xs - margin) / P.cw[0]);
            int xhi = (int)floor((xs + margin) / P.cw[0]);
            if (all_y || xhi - xlo + 1 >= P.nc[0]) { xlo = 0; xhi = P.nc[0] - 1; }
            for (int xc = xlo; xc <= xhi; ++xc) {
                const int xx = ((xc % P.nc[0]) + P.nc[0]) % P.nc[0];
                const uint32_t key = cell_key(P, xx, yy, zz);
                const uint32_t st = b.cell_start[key], en = st + b.cell_cnt[key];
                for (uint32_t j = st; j < en; ++j) {
                    if (!(idi < b.id[j])) continue;
                    double dx, dy, dz;
                    min_image(P, s_le, pi, b.pos[j], dx, dy, dz);
                    rdf_bin(dx, dy, dz, mode, r_max, slab, nbins, counts);
                }
            }
        }
    }
}

void launch_rdf(const Bufs& b, hipStream_t st, int p, uint32_t rep, uint32_t nblk, int mode, double r_max,
                double slab, double reach, uint32_t nbins, unsigned long long* counts) {
    hipLaunchKernelGGL(k_rdf, dim3(nblk), dim3(256), 0, st, b, rep, p, mode, r_max, slab, reach, nbins, counts);
}

// Scratch memory of the entry points that allocate nothing: a file-scope device
// array (one copy per GPU, held until the process ends).  Host code never uses the
// array's name as an address: each device's copy is looked up once, with that device
// current, by hipGetSymbolAddress, and that pointer is what kernels and copies get.
static __device__ __align__(256) unsigned long long scratch[kScratchWords];

unsigned long long* scratch_ptr(std::string& err) {
    static std::mutex mu;
    static unsigned long long* ptrs[kMaxDevices] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        err = "no current device (or its index is beyond the supported range)";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptrs[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e);
            return nullptr;
        }
        ptrs[dev] = (unsigned long long*)p;
    }
    return ptrs[dev];
}

// zeroes n 64-bit words (a kernel, not a memset node, so that the call can sit in
// a captured graph)
__global__ __launch_bounds__(256) void k_zero64(unsigned long long* a, uint32_t n) {
    for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) a[k] = 0ull;
}

void launch_zero64(hipStream_t st, unsigned long long* a, uint32_t n) {
    const uint32_t g = std::min<uint32_t>((n + 255) / 256, 1024u);
    hipLaunchKernelGGL(k_zero64, dim3(g), dim3(256), 0, st, a, n);
}

// Time autocorrelation of recorded stress component comp (0..26) of one
// replica: one block per lag, a fixed-order sum over the record pairs.
__global__ __launch_bounds__(256) void k_acf(Bufs b, uint32_t rep, int comp, uint32_t first, uint32_t count,
                                             double* out) {
    const uint32_t lag = blockIdx.x;
    const double* ring = b.ring + (size_t)rep * kRing * 27;
    double acc = 0.0;
    for (uint32_t t = threadIdx.x; t + lag < count; t += blockDim.x) {
        const uint32_t s0 = (first + t) % kRing, s1 = (first + t + lag) % kRing;
        acc += ring[(size_t)s0 * 27 + comp] * ring[(size_t)s1 * 27 + comp];
    }
    __shared__ double rows[16];
    acc = row_sum_f64(acc);
    if ((threadIdx.x & 15) == 15) rows[threadIdx.x >> 4] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 4); ++k) t += rows[k];
        out[lag] = lag < count ? t / (double)(count - lag) : 0.0;
    }
}

void launch_acf(const Bufs& b, hipStream_t st, uint32_t rep, int comp, uint32_t first, uint32_t count,
                uint32_t nlag, double* out) {
    hipLaunchKernelGGL(k_acf, dim3(nlag), dim3(256), 0, st, b, rep, comp, first, count, out);
}

// Structural Brownian stress sum of one replica (Sec. II.D) at parity p:
// per particle i, (a_i / Delta_i) n n over its list partners with gap
// h <= Delta_i = 0.05 a_i, in list (id) order; part[block * 9 + c] receives
// the block's fixed-order sum.  The caller scales by -kT / V.
__global__ __launch_bounds__(256) void k_struct(Bufs b, uint32_t rep, int p, double* part) {
    const RepParams& P = b.reps[rep];
    const uint32_t i = P.p_begin + blockIdx.x * 256 + threadIdx.x;
    double acc[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] = 0.0;
    if (i - P.p_begin < P.n) {
        const double4 pi = b.pos[i];
        const double s_le = b.dyn[rep].s_slot[p];
        const double delta = 0.05 * pi.w, wgt = pi.w / delta;
        const uint32_t cnt = b.ncnt[i];
        for (uint32_t e = 0; e < cnt; ++e) {
            const double4 pj = b.pos[b.nbr[e * b.npad + i]];
            double r[3];
            min_image(P, s_le, pi, pj, r[0], r[1], r[2]);
            const double dist = sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
            if (!(dist - (pi.w + pj.w) <= delta)) continue;
#pragma unroll
            for (int al = 0; al < 3; ++al)
#pragma unroll
                for (int be = 0; be < 3; ++be) acc[3 * al + be] += wgt * (r[al] / dist) * (r[be] / dist);
        }
    }
    __shared__ double rows[16][9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const double v = row_sum_f64(acc[c]);
        if ((threadIdx.x & 15) == 15) rows[threadIdx.x >> 4][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += rows[k][threadIdx.x];
        part[blockIdx.x * 9 + threadIdx.x] = t;
    }
}

void launch_struct(const Bufs& b, hipStream_t st, int p, uint32_t rep, uint32_t nblk, double* part) {
    hipLaunchKernelGGL(k_struct, dim3(nblk), dim3(256), 0, st, b, rep, p, part);
}

// diagnostics: mode 0 = interaction set, 1 = Verlet list, 2 = contacts (with springs)
__global__ void k_diag(Bufs b, int p, uint32_t rep, uint32_t* out_ij, double* out_s, int32_t* out_sl,
                       uint32_t* count, uint32_t cap, int mode) {
    const RepParams& P = b.reps[rep];
    const uint32_t i = P.p_begin + blockIdx.x * blockDim.x + threadIdx.x;
    if (i - P.p_begin >= P.n) return;
    const double4 pi = b.pos[i];
    const uint32_t idi = b.id[i];
    const uint32_t cnt = b.ncnt[i];
    const uint64_t cm = b.cmask[i], sm = b.smask[i];
    const double s_le = b.dyn[rep].s_slot[p];
    for (uint32_t e = 0; e < cnt; ++e) {
        const uint32_t j = b.nbr[e * b.npad + i];
        const uint32_t idj = b.id[j];
        if (!(idi < idj)) continue;
        bool take;
        if (mode == 1) {
            take = true;
        } else if (mode == 2) {
            take = (cm >> e) & 1ull;
        } else {
            double dx, dy, dz;
            min_image(P, s_le, pi, b.pos[j], dx, dy, dz);
            const double d2 = (dx * dx + dy * dy) + dz * dz;
            const double rc = (pi.w + b.pos[j].w) * P.c1;
            take = d2 <= rc * rc;
        }
        if (!take) continue;
        const uint32_t k = atomicAdd(count, 1u);
        if (k < cap) {
            out_ij[2 * k] = idi;
            out_ij[2 * k + 1] = idj;
            if (mode == 2) {
                spring_f64(b, e * b.npad + i, out_s + 3 * k);
                out_sl[k] = (int32_t)((sm >> e) & 1ull);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline uint32_t nblocks(uint32_t n, uint32_t bs) { return (n + bs - 1) / bs; }

void launch_integrate(const Bufs& b, hipStream_t st, int q) {
    if (b.mixed) hipLaunchKernelGGL(k_integrate<true>, dim3(b.npad / 256), dim3(256), 0, st, b, q);
    else hipLaunchKernelGGL(k_integrate<false>, dim3(b.npad / 256), dim3(256), 0, st, b, q);
}

void launch_finalize(const Bufs& b, hipStream_t st, int q) {
    hipLaunchKernelGGL(k_finalize, dim3(27 * b.nrep), dim3(256), 0, st, b, q);
}

void launch_rebuild(const Bufs& b, hipStream_t st, int q, int in_step, uint32_t ct_input_rep) {
    const uint32_t np = b.npad / 256;
    hipLaunchKernelGGL(k_rb_zero, dim3(nblocks(b.nkeys_total, 256)), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_rb_keys, dim3(np), dim3(256), 0, st, b);
    const uint32_t nsb = nblocks(b.nkeys_total, kScanTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nsb), dim3(kScanBlock), 0, st, b);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, st, b, nsb);
    hipLaunchKernelGGL(k_scan_down, dim3(nsb), dim3(kScanBlock), 0, st, b);
    hipLaunchKernelGGL(k_rb_scatter, dim3(np), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_rb_cellsort, dim3(nblocks(b.nkeys_total, 256)), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_rb_gather, dim3(np), dim3(256), 0, st, b, ct_input_rep);
    hipLaunchKernelGGL(k_rb_copyback, dim3(np), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_rb_need0, dim3(1), dim3(64), 0, st, b);
    hipLaunchKernelGGL(k_rb_nlist, dim3(np), dim3(256), 0, st, b, q, in_step);
    hipLaunchKernelGGL(k_rb_mirror, dim3(np), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_rb_reset, dim3(1), dim3(256), 0, st, b, q);
}

void launch_relist(const Bufs& b, hipStream_t st, int q, int in_step) {
    const uint32_t np = b.npad / 256;
    hipLaunchKernelGGL(k_rb_need0, dim3(1), dim3(64), 0, st, b);
    hipLaunchKernelGGL(k_rb_nlist, dim3(np), dim3(256), 0, st, b, q, in_step);
    hipLaunchKernelGGL(k_rb_mirror, dim3(np), dim3(256), 0, st, b);
}

// One launch, or with ev (start, stop) a launch whose events are recorded by the
// hardware when the kernel starts and ends (the profiled pass times kernels so).
template <typename F, typename... Args>
static void launch_k(F kern, dim3 grid, dim3 blk, hipStream_t st, const hipEvent_t* ev, Args... args) {
    if (ev) hipExtLaunchKernelGGL(kern, grid, blk, 0, st, ev[0], ev[1], 0u, args...);
    else hipLaunchKernelGGL(kern, grid, blk, 0, st, args...);
}

template <bool MIX>
static void launch_pair_t(const Bufs& b, hipStream_t st, int q, int kick, int advance, uint32_t only_rep,
                          const hipEvent_t* kev, int fuse) {
    const hipEvent_t* ev0 = kev;                        // pair kernel
    const hipEvent_t* ev1 = kev ? kev + 2 : nullptr;    // gather
    // half-pair evaluation, then the per-particle gather
    const uint32_t g = b.npad / 256, fin = (27u * b.nrep + 7u) & ~7u;  // finalize blocks, then pair blocks
    if (b.ext) {
        switch (b.lanes) {
            case 1: launch_k(k_half<MIX, 1, true>, dim3(g + fin), dim3(256), st, ev0, b, q, advance, only_rep); break;
            case 2: launch_k(k_half<MIX, 2, true>, dim3(2 * g + fin), dim3(256), st, ev0, b, q, advance, only_rep); break;
            default: launch_k(k_half<MIX, 4, true>, dim3(4 * g + fin), dim3(256), st, ev0, b, q, advance, only_rep); break;
        }
    } else if (!MIX && b.occ) {
        switch (b.lanes) {
            case 1: launch_k(k_half<false, 1, false, true>, dim3(g + fin), dim3(256), st, ev0, b, q, advance, only_rep); break;
            case 2: launch_k(k_half<false, 2, false, true>, dim3(2 * g + fin), dim3(256), st, ev0, b, q, advance, only_rep); break;
            default: launch_k(k_half<false, 4, false, true>, dim3(4 * g + fin), dim3(256), st, ev0, b, q, advance, only_rep); break;
        }
    } else {
        switch (b.lanes) {
            case 1: launch_k(k_half<MIX, 1, false>, dim3(g + fin), dim3(256), st, ev0, b, q, advance, only_rep); break;
            case 2: launch_k(k_half<MIX, 2, false>, dim3(2 * g + fin), dim3(256), st, ev0, b, q, advance, only_rep); break;
            default: launch_k(k_half<MIX, 4, false>, dim3(4 * g + fin), dim3(256), st, ev0, b, q, advance, only_rep); break;
        }
    }
    if (b.rot) launch_k(k_gather<MIX, true>, dim3(b.npad / 256), dim3(256), st, ev1, b, q, kick, fuse, only_rep);
    else launch_k(k_gather<MIX, false>, dim3(b.npad / 256), dim3(256), st, ev1, b, q, kick, fuse, only_rep);
}

void launch_pair_force(const Bufs& b, hipStream_t st, int q, int kick, int advance, uint32_t only_rep,
                       const hipEvent_t* kev, int fuse) {
    if (b.mixed) launch_pair_t<true>(b, st, q, kick, advance, only_rep, kev, fuse);
    else launch_pair_t<false>(b, st, q, kick, advance, only_rep, kev, fuse);
}

void launch_diag(const Bufs& b, hipStream_t st, int p, uint32_t rep, uint32_t n, uint32_t* out_ij, double* out_s,
                 int32_t* out_sl, uint32_t* count, uint32_t cap, int mode) {
    hipLaunchKernelGGL(k_diag, dim3(nblocks(n, 256)), dim3(256), 0, st, b, p, rep, out_ij, out_s, out_sl, count, cap,
                       mode);
}

}  // namespace susp
