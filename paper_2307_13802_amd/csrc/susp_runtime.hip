// Host runtime and C ABI of the force engine (declared in include/sim.h):
// configuration checks, device memory, the per-step launch sequence captured
// in HIP graphs, state transfer in particle-id order and diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sim.h"
#include "susp.h"

using namespace susp;

namespace {

std::mutex g_mu;
std::string g_err;  // message of the last failure not tied to a handle
void* (*g_alloc)(size_t, void*) = nullptr;
void (*g_free)(void*, void*) = nullptr;
void* g_alloc_ctx = nullptr;

constexpr uint32_t kDefaultCap = 48;
constexpr uint32_t kMaxCap = 64;     // list entries per particle: the width of the entry bit masks
// Verlet skin of a replica: the configured one, or (skin <= 0) skin_frac times the
// smallest radius (0.2 by default; the tuner chooses among kSkinFracs for skin < 0)
constexpr double kSkinDefault = 0.2;
constexpr double kSkinFracs[] = {0.1, 0.15, 0.2, 0.3, 0.4};
constexpr double kCellFactors[] = {1.0, 1.5, 2.0};
constexpr double kRepRange = 16.0;   // the repulsion acts up to a gap of 16 kappa, kappa = 0.01 (a_i + a_j)

// Tunable launch and list parameters (one set per handle).  None of them changes a
// trajectory: each particle's force is summed over its interacting partners in id
// order whatever the lanes per particle, the kernel form, the skin of the list or the
// cell size of the layout.  The stress sums run over pairs in an order that follows
// the launch shape, so their last bits can differ between parameter sets.
struct Tune {
    int lanes = 1, occ = 0;
    double skin_frac = kSkinDefault;  // skin = skin_frac * a_min (when not configured)
    double cell = 1.0;                // search cells at least cell * list range wide
    int source = 0;                   // 0 configured / default, 1 measured, 2 cache
};

constexpr int kGraphSteps = 8;     // step graphs of kGraphLong, kGraphSteps and 1 steps
constexpr int kGraphLong = 64;

struct HipError {
    hipError_t e;
    const char* what;
};

#define HIPCHK(x)                                        \
    do {                                                 \
        hipError_t e__ = (x);                            \
        if (e__ != hipSuccess) throw HipError{e__, #x};  \
    } while (0)

void set_global_error(const std::string& m) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_err = m;
}

std::string fmt(const char* f, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof buf, f, ap);
    va_end(ap);
    return buf;
}

}  // namespace

struct sim {
    int nrep = 0;
    int mixed = 0;
    uint32_t flags = 0;
    std::vector<sim_config> cfg;
    std::vector<std::vector<double>> radii;  // id order
    std::vector<RepParams> P;
    std::vector<double> drag_xy;             // drag stresslet sigma_xy = sigma_yx per replica
    std::vector<uint32_t> ring_tail;
    Bufs b{};
    hipStream_t st = nullptr;
    hipStream_t cap_st = nullptr;            // stream used only to capture graphs
    // step graphs [1 | kGraphSteps | kGraphLong steps][parity of the first step][integrates first]
    // [hands over fused]
    hipGraphExec_t gc[3][2][2][2] = {};
    std::vector<std::pair<void*, size_t>> allocs;
    void* (*afn)(size_t, void*) = nullptr;
    void (*ffn)(void*, void*) = nullptr;
    void* actx = nullptr;
    std::string err;
    int profile = 0;
    std::vector<hipEvent_t> ev;
    int64_t prof_launches = 0;
    double prof_ms = 0.0;
    double prof_stage_ms[3] = {0.0, 0.0, 0.0};  // integrate, pair kernel, gather
    int64_t steps_total = 0;
    uint64_t step_now = 0;       // step counter of replica 0 (all replicas advance together)
    int par = 0;                 // parity of the current state (slot of the last evaluation)
    int64_t since_build = 0;     // steps since the last list build
    int64_t plan = 16;           // rebuild when since_build reaches this
    int64_t plan_hint = 16;      // first chunk after a build
    double* struct_part = nullptr;  // block sums of the structural Brownian stress
    uint32_t struct_cap = 0;
    uint32_t keys_cap = 0;       // cell keys allocated (the finest layout a parameter set can ask for)
    std::vector<RepDyn> dyn_host;  // host copy of the per-replica records read by the health check
    int short_q = -1;            // >= 0: the last build found lists too short; regrow and build them
                                 // again (parity q) before they are used
    uint32_t short_need = 0;     // the largest partner count it found
    std::string list_fail;       // a list that cannot grow enough (reported by the health check)
    Tune tune;                   // parameter set in use

    void* dalloc(size_t bytes) {
        if (bytes == 0) bytes = 256;
        void* p = nullptr;
        if (afn) {
            p = afn(bytes, actx);
            if (!p) throw HipError{hipErrorOutOfMemory, "allocator hook"};
        } else {
            HIPCHK(hipMalloc(&p, bytes));
        }
        allocs.push_back({p, bytes});
        HIPCHK(hipMemsetAsync(p, 0, bytes, st));
        return p;
    }
    template <class T> T* alloc(size_t count) { return (T*)dalloc(count * sizeof(T)); }
    // frees one allocation made by dalloc (after the stream's work on it)
    void release(void* p) {
        for (size_t k = 0; k < allocs.size(); ++k)
            if (allocs[k].first == p) {
                (void)hipStreamSynchronize(st);
                if (ffn) ffn(p, actx);
                else (void)hipFree(p);
                allocs.erase(allocs.begin() + (long)k);
                return;
            }
    }

    ~sim() {
        for (auto& a : gc)
            for (auto& b2 : a)
                for (auto& c : b2)
                    for (auto& g : c)
                        if (g) (void)hipGraphExecDestroy(g);
        for (auto& e : ev) (void)hipEventDestroy(e);
        (void)hipStreamSynchronize(st);
        for (auto& a : allocs) {
            if (ffn) ffn(a.first, actx);
            else (void)hipFree(a.first);
        }
        if (cap_st) (void)hipStreamDestroy(cap_st);
    }
};

namespace {

int fail(sim* s, int code, const std::string& m) {
    if (s) s->err = m;
    else set_global_error(m);
    return code;
}

int hip_fail(sim* s, const HipError& e) {
    return fail(s, SIM_EDEVICE, fmt("%s failed: %s", e.what, hipGetErrorString(e.e)));
}

double min_radius(const double* a, uint32_t n) {
    double m = a[0];
    for (uint32_t i = 1; i < n; ++i) m = std::min(m, a[i]);
    return m;
}

double max_radius(const double* a, uint32_t n) {
    double m = a[0];
    for (uint32_t i = 1; i < n; ++i) m = std::max(m, a[i]);
    return m;
}


double eff_skin(const sim_config& c, const double* radii, double frac) {
    return c.skin > 0.0 ? c.skin : frac * min_radius(radii, c.n);
}

// range factor of the pairs evaluated: the lubrication cut-off, or the repulsion's range
double range_factor(const sim_config& c) {
    const double c1 = 1.0 + 0.5 * c.xi_cut;
    const double cr = 1.0 + kRepRange * 0.01;
    return c.repulsion > 0.0 && cr > c1 ? cr : c1;
}

// the minimum image is unique when every box side exceeds twice the list range
bool box_fits(const sim_config& c, const double* radii, double skin) {
    const double rl = 2.0 * max_radius(radii, c.n) * range_factor(c) + skin;
    for (int d = 0; d < 3; ++d)
        if (!(c.box[d] > 2.0 * rl)) return false;
    return true;
}

int validate(const sim_config* c, const double* radii, std::string& why) {
    if (!c) { why = "null config"; return SIM_EINVAL; }
    if (c->struct_size != sizeof(sim_config)) {
        why = fmt("struct_size %u != sizeof(sim_config) %zu", c->struct_size, sizeof(sim_config));
        return SIM_EINVAL;
    }
    if (c->lanes != 0 && c->lanes != 1 && c->lanes != 2 && c->lanes != 4) {
        why = "lanes must be 0, 1, 2 or 4";
        return SIM_EINVAL;
    }
    if (c->pair_kernel != SIM_KERNEL_AUTO && c->pair_kernel != SIM_KERNEL_HALF) {
        why = "pair_kernel must be SIM_KERNEL_AUTO or SIM_KERNEL_HALF";
        return SIM_EINVAL;
    }
    if ((c->flags & SIM_HALF_OCC_ON) && (c->flags & SIM_HALF_OCC_OFF)) {
        why = "SIM_HALF_OCC_ON and SIM_HALF_OCC_OFF exclude each other";
        return SIM_EINVAL;
    }
    if ((c->flags & SIM_HALF_OCC_ON) && (c->precision != SIM_FP64 || (c->flags & SIM_LUB_ROT) || c->repulsion > 0.0)) {
        why = "SIM_HALF_OCC_ON needs FP64 and no model switch";
        return SIM_EINVAL;
    }
    if (c->reserved != 0) { why = "reserved field must be 0"; return SIM_EINVAL; }
    if (!(c->cell_factor == 0.0 || c->cell_factor < 0.0 || (c->cell_factor >= 1.0 && c->cell_factor <= 4.0))) {
        why = "cell_factor must be 0 (1.0), negative (tuned) or in [1, 4]";
        return SIM_EINVAL;
    }
    if (c->n == 0 || c->n >= 0xFFFFFFFFu) { why = "n must be in [1, 2^32-2]"; return SIM_EINVAL; }
    if (!radii) { why = "null radii"; return SIM_EINVAL; }
    for (uint32_t i = 0; i < c->n; ++i)
        if (!(radii[i] > 0.0) || !std::isfinite(radii[i])) { why = fmt("radius %u is not positive", i); return SIM_EINVAL; }
    for (int d = 0; d < 3; ++d)
        if (!(c->box[d] > 0.0) || !std::isfinite(c->box[d])) { why = "box sides must be positive"; return SIM_EINVAL; }
    if (!(c->dt > 0.0)) { why = "dt must be positive"; return SIM_EINVAL; }
    if (!(c->rho > 0.0) || !(c->eta > 0.0)) { why = "rho and eta must be positive"; return SIM_EINVAL; }
    if (c->kn < 0.0 || c->kt < 0.0 || c->mu < 0.0 || c->kT < 0.0 || !(c->repulsion >= 0.0)) {
        why = "kn, kt, mu, kT and repulsion must be non-negative";
        return SIM_EINVAL;
    }
    if (!std::isfinite(c->gammadot)) { why = "gammadot must be finite"; return SIM_EINVAL; }
    if (!(c->xi_min > 0.0) || !(c->xi_min < c->xi_cut)) { why = "need 0 < xi_min < xi_cut"; return SIM_EINVAL; }
    if (c->precision != SIM_FP64 && c->precision != SIM_MIXED) { why = "unknown precision"; return SIM_EINVAL; }
    if (c->nlist_cap > 64) { why = "nlist_cap must be <= 64"; return SIM_EINVAL; }
    // with a tuned skin the smallest candidate must fit
    const double skin = eff_skin(*c, radii, c->skin < 0.0 ? kSkinFracs[0] : kSkinDefault);
    if (!box_fits(*c, radii, skin)) {
        const double rl = 2.0 * max_radius(radii, c->n) * range_factor(*c) + skin;
        why = fmt("every box side must exceed twice the list range %g", rl);
        return SIM_EINVAL;
    }
    return SIM_OK;
}

int key_bits(int n) {
    int b = 0;
    while ((1 << b) < n) ++b;
    return b;
}

// host copy of one replica's slots [p_begin, p_begin + n_pad)
template <class T> std::vector<T> d2h(sim* s, const T* dev, size_t off, size_t count) {
    std::vector<T> h(count);
    HIPCHK(hipMemcpyAsync(h.data(), dev + off, count * sizeof(T), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return h;
}

// Destroys the captured step graphs (they are captured again on the next step).
void drop_graphs(sim* s) {
    for (auto& a : s->gc)
        for (auto& b2 : a)
            for (auto& c : b2)
                for (auto& g : c)
                    if (g) {
                        (void)hipGraphExecDestroy(g);
                        g = nullptr;
                    }
}

// Regrows the per-entry arrays of the lists (partners, springs, mirror index, pair
// records) to hold `need` entries per particle, and builds the lists again from the
// cells and the carried contact history of the build just done (which stay valid
// until the next build).  Beyond kMaxCap entries (or 2^32 list slots) the lists
// cannot grow: the failure is left for the health check to report.
void regrow_lists(sim* s, int q, int in_step, uint32_t need) {
    Bufs& b = s->b;
    const size_t np = b.npad;
    const uint32_t cap = std::min(kMaxCap, (need + 7u) & ~7u);
    if (need > kMaxCap || (uint64_t)np * cap >= (1ull << 32)) {
        s->list_fail = fmt("a particle has %u partners within the list range; the lists hold at most %u", need,
                           need > kMaxCap ? kMaxCap : b.cap);
        return;
    }
    const size_t rs = s->mixed ? sizeof(float) : sizeof(double);
    const size_t recs = s->mixed ? 4 * sizeof(float) : 3 * sizeof(double);
    // the new arrays first, so that a failed allocation leaves the handle's lists as they were
    void* const old[6] = {b.nbr, b.hs, b.mir, b.pf, b.pt, b.pt2};
    void* nw[6] = {};
    try {
        nw[0] = s->dalloc(np * cap * sizeof(uint32_t));
        nw[1] = s->dalloc(np * cap * 3 * rs);
        nw[2] = s->dalloc(np * cap);
        nw[3] = s->dalloc(np * cap * recs);
        nw[4] = s->dalloc(np * cap * recs);
        nw[5] = s->dalloc(np * cap * recs);
    } catch (...) {
        for (void* p : nw)
            if (p) s->release(p);
        throw;
    }
    b.nbr = (uint32_t*)nw[0];
    b.hs = nw[1];
    b.mir = (uint8_t*)nw[2];
    b.pf = nw[3];
    b.pt = nw[4];
    b.pt2 = nw[5];
    for (void* p : old) s->release(p);
    b.cap = cap;
    drop_graphs(s);   // captured launches hold the buffer table by value
    launch_relist(b, s->st, q, in_step);
    HIPCHK(hipGetLastError());
}

// A list build of parity q (launch_rebuild), then the regrow when it found a particle
// with more partners than the lists hold.  grow false (a caller that cannot allocate):
// the regrow waits for the next call that uses the lists (ensure_lists).  in_step
// builds (those between kick 1 and the forces of a step) are always regrown at once.
void rebuild(sim* s, int q, int in_step, uint32_t ct_input_rep, bool grow = true) {
    launch_rebuild(s->b, s->st, q, in_step, ct_input_rep);
    uint32_t need = 0;
    HIPCHK(hipMemcpyAsync(&need, (char*)s->b.sys + offsetof(SysDyn, list_need), sizeof need,
                          hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    s->short_q = -1;
    if (need == 0) return;
    if (!grow && !in_step) {
        s->short_q = q;
        s->short_need = need;
        return;
    }
    regrow_lists(s, q, in_step, need);
}

// Regrows lists that a build without allocation left short (before they are used).
void ensure_lists(sim* s) {
    if (s->short_q < 0) return;
    const int q = s->short_q;
    s->short_q = -1;
    regrow_lists(s, q, 0, s->short_need);
}

// nsteps time steps, the first with parity q0, without a list rebuild; every
// launch does nothing once the expiry test of an earlier one has halted the
// chunk.  With the half-pair variant the gather of each step but the last
// also takes kick 1 and the drift of the next step.
// With the half-pair kernel a step's gather also takes kick 1 and the drift of
// the next step (fused), so only the first step of a launch sequence integrates
// and only its last leaves the full-step values in memory.  integrate_first:
// this run of steps starts a sequence; fuse_last: it does not end one (the next
// run continues it without an integrate).
void enqueue_steps(sim* s, hipStream_t st, int nsteps, int q0, bool integrate_first = true, bool fuse_last = false) {
    for (int k = 0; k < nsteps; ++k) {
        const int q = q0 ^ (k & 1);
        if (k == 0 && integrate_first) launch_integrate(s->b, st, q);
        launch_pair_force(s->b, st, q, 1, 1, 0xFFFFFFFFu, nullptr, k + 1 < nsteps || fuse_last);
    }
}

hipGraphExec_t capture(sim* s, int nsteps, int q0, bool integrate_first, bool fuse_last) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIPCHK(hipStreamBeginCapture(s->cap_st, hipStreamCaptureModeThreadLocal));
    enqueue_steps(s, s->cap_st, nsteps, q0, integrate_first, fuse_last);
    HIPCHK(hipStreamEndCapture(s->cap_st, &g));
    HIPCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    HIPCHK(hipGraphDestroy(g));
    return ge;
}

// Reads and clears the health flags; returns a status.
int check_health(sim* s) {
    std::vector<RepDyn>& dyn = s->dyn_host;   // sized at creation: no allocation here
    HIPCHK(hipMemcpyAsync(dyn.data(), s->b.dyn, sizeof(RepDyn) * s->nrep, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    int code = SIM_OK;
    std::string msg;
    if (!s->list_fail.empty()) {
        code = SIM_ECAPACITY;
        msg = s->list_fail;
        s->list_fail.clear();
    }
    for (int r = 0; r < s->nrep; ++r) {
        const uint32_t h = dyn[r].health;
        if (!h) continue;
        if ((h & H_NLIST) && code != SIM_ECAPACITY) {
            code = SIM_ECAPACITY;
            msg = fmt("replica %d: neighbour list or contact capacity exceeded at step %llu", r,
                      (unsigned long long)std::max(dyn[r].step_slot[0], dyn[r].step_slot[1]));
        } else if (code == SIM_OK) {
            code = SIM_EUNSTABLE;
            msg = fmt("replica %d: %s at step %llu", r, (h & H_NAN) ? "non-finite force" : "overlap above the limit",
                      (unsigned long long)std::max(dyn[r].step_slot[0], dyn[r].step_slot[1]));
        }
        const uint32_t zero = 0;
        HIPCHK(hipMemcpyAsync((char*)(s->b.dyn + r) + offsetof(RepDyn, health), &zero, sizeof zero,
                              hipMemcpyHostToDevice, s->st));
    }
    HIPCHK(hipStreamSynchronize(s->st));
    if (code != SIM_OK) s->err = msg;
    return code;
}

// Writes the state of replica r (id order) into its slots, and its contact
// history into the host-input half of the compact table.
void upload_state(sim* s, int r, const double* x, const double* v, const double* w, const double* F,
                  const double* T, const uint32_t* cij, const double* cs, int64_t nc) {
    const RepParams& P = s->P[r];
    const uint32_t n = P.n, np = P.n_pad, p0 = P.p_begin, npad = s->b.npad;
    const std::vector<double>& a = s->radii[r];
    std::vector<double4> pos(np), vv(np), ww(np), FF(np), TT(np);
    std::vector<float4> vs(np), ws(np), Ff(np), Tf(np);
    std::vector<uint32_t> id(np, kNoId);
    for (uint32_t i = 0; i < n; ++i) {
        pos[i] = make_double4(x[3 * i], x[3 * i + 1], x[3 * i + 2], a[i]);
        const double* vi = v ? v + 3 * i : nullptr;
        double vx = vi ? vi[0] : P.gd * (x[3 * i + 1] - 0.5 * P.L[1]);
        vv[i] = make_double4(vx, vi ? vi[1] : 0.0, vi ? vi[2] : 0.0, 0.0);
        ww[i] = w ? make_double4(w[3 * i], w[3 * i + 1], w[3 * i + 2], 0.0) : make_double4(0.0, 0.0, -0.5 * P.gd, 0.0);
        FF[i] = F ? make_double4(F[3 * i], F[3 * i + 1], F[3 * i + 2], 0.0) : make_double4(0, 0, 0, 0);
        TT[i] = T ? make_double4(T[3 * i], T[3 * i + 1], T[3 * i + 2], 0.0) : make_double4(0, 0, 0, 0);
        vs[i] = make_float4((float)vv[i].x, (float)vv[i].y, (float)vv[i].z, 0.f);
        ws[i] = make_float4((float)ww[i].x, (float)ww[i].y, (float)ww[i].z, 0.f);
        Ff[i] = make_float4((float)FF[i].x, (float)FF[i].y, (float)FF[i].z, 0.f);
        Tf[i] = make_float4((float)TT[i].x, (float)TT[i].y, (float)TT[i].z, 0.f);
        id[i] = i;
    }
    // compact contact table (both sides of each contact), host-input half; checked before
    // anything is uploaded, so that a rejected state leaves the replica as it was
    std::vector<uint32_t> cnt(np, 0), cid((size_t)kCtCap * np, 0);
    std::vector<double> cvs((size_t)kCtCap * 3 * np, 0.0);
    for (int64_t k = 0; k < nc; ++k) {
        const uint32_t i = cij[2 * k], j = cij[2 * k + 1];
        if (i >= n || j >= n || i == j) throw std::string(fmt("contact %lld has invalid ids (%u, %u)", (long long)k, i, j));
        if (!(i < j)) throw std::string(fmt("contact %lld must list the lower id first", (long long)k));
        for (int side = 0; side < 2; ++side) {
            const uint32_t me = side ? j : i, other = side ? i : j;
            if (cnt[me] >= (uint32_t)kCtCap) throw std::string(fmt("particle %u has more than %d contacts", me, kCtCap));
            const uint32_t c = cnt[me]++;
            cid[(size_t)c * np + me] = other;
            for (int d = 0; d < 3; ++d) cvs[((size_t)c * 3 + d) * np + me] = cs[3 * k + d];
        }
    }
    hipStream_t st = s->st;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    };
    up(s->b.pos + p0, pos.data(), np * sizeof(double4));
    up(s->b.vh + p0, vv.data(), np * sizeof(double4));
    up(s->b.vf + p0, vv.data(), np * sizeof(double4));
    up(s->b.wh + p0, ww.data(), np * sizeof(double4));
    up(s->b.wf + p0, ww.data(), np * sizeof(double4));
    up(s->b.id + p0, id.data(), np * sizeof(uint32_t));
    if (s->mixed) {
        up(s->b.vsh + p0, vs.data(), np * sizeof(float4));
        up(s->b.wsh + p0, ws.data(), np * sizeof(float4));
        up((float4*)s->b.F + p0, Ff.data(), np * sizeof(float4));
        up((float4*)s->b.T + p0, Tf.data(), np * sizeof(float4));
    } else {
        up((double4*)s->b.F + p0, FF.data(), np * sizeof(double4));
        up((double4*)s->b.T + p0, TT.data(), np * sizeof(double4));
    }
    up(s->b.ct_n + npad + p0, cnt.data(), np * sizeof(uint32_t));
    for (int c = 0; c < kCtCap; ++c) {
        up(s->b.ct_id + (size_t)(kCtCap + c) * npad + p0, cid.data() + (size_t)c * np, np * sizeof(uint32_t));
        for (int d = 0; d < 3; ++d)
            up(s->b.ct_s + ((size_t)(kCtCap + c) * 3 + d) * npad + p0, cvs.data() + ((size_t)c * 3 + d) * np,
               np * sizeof(double));
    }
    // its displacement record starts again
    HIPCHK(hipMemsetAsync(s->b.disp + p0, 0, np * sizeof(double4), st));
    // list of this replica becomes invalid; its history now comes from the table
    HIPCHK(hipMemsetAsync(s->b.ncnt + p0, 0, np * sizeof(uint32_t), st));
    HIPCHK(hipMemsetAsync(s->b.cmask + p0, 0, np * sizeof(uint64_t), st));
    HIPCHK(hipMemsetAsync(s->b.smask + p0, 0, np * sizeof(uint64_t), st));
}

void set_dyn(sim* s, int r, double s_le, uint64_t step) {
    RepDyn d{};
    d.s_slot[0] = d.s_slot[1] = s_le;
    d.step_slot[0] = d.step_slot[1] = step;
    HIPCHK(hipMemcpyAsync(s->b.dyn + r, &d, sizeof d, hipMemcpyHostToDevice, s->st));
    s->ring_tail[r] = 0;
}

void set_variant(sim* s, int lanes, int occ) {
    s->b.lanes = lanes;
    s->b.occ = occ;
    s->b.ppb = 256 / lanes;
}

// Per-replica parameters for a skin fraction and cell factor; p_begin, blocks and
// key offsets are filled by the caller.
RepParams rep_params(const sim_config& c, const double* radii, double skin_frac, double cell) {
    RepParams P{};
    for (int d = 0; d < 3; ++d) {
        P.L[d] = c.box[d];
        P.invL[d] = 1.0 / c.box[d];
    }
    P.gd = c.gammadot;
    P.gdLy = c.gammadot * c.box[1];
    P.dt = c.dt;
    P.half_dt = 0.5 * c.dt;
    P.rho = c.rho; P.eta = c.eta; P.kn = c.kn; P.kt = c.kt; P.mu = c.mu;
    P.rep_A = c.repulsion;
    P.kT = c.kT;
    P.bamp = std::sqrt(2.0 * c.kT / c.dt);
    P.c1 = 1.0 + 0.5 * c.xi_cut;
    P.c_int = range_factor(c);
    P.xi_min = c.xi_min;
    P.skin = eff_skin(c, radii, skin_frac);
    const double amax = max_radius(radii, c.n), amin = min_radius(radii, c.n);
    P.rc_max = 2.0 * amax * P.c_int;
    P.rl_max = P.rc_max + P.skin;
    P.invV = 1.0 / (c.box[0] * c.box[1] * c.box[2]);
    const double cf = c.cell_factor > 0.0 ? c.cell_factor : cell;
    int mx = 1;
    for (int d = 0; d < 3; ++d) {
        int nc = (int)std::floor(c.box[d] / (P.rl_max * cf));
        if (nc < 3) nc = 1;
        if (nc > 1024) nc = 1024;
        P.nc[d] = nc;
        P.cw[d] = c.box[d] / nc;
        mx = std::max(mx, nc);
    }
    P.mbits = key_bits(mx);
    P.nkeys = (1u << (3 * P.mbits)) + 1u;
    P.max_overlap = c.max_overlap > 0.0 ? c.max_overlap : 0.1 * amin;
    P.n = c.n;
    P.n_pad = (c.n + kTile - 1) / kTile * kTile;
    P.flags = c.flags;
    P.nblk = P.n_pad / kTile;
    P.seed = c.seed;
    return P;
}

// Parameter table of every replica for one parameter set (key offsets laid out in
// replica order); total cell keys in *keys.
std::vector<RepParams> layout(const sim* s, const Tune& t, uint32_t* keys) {
    std::vector<RepParams> out;
    uint32_t p = 0, key = 0;
    for (int r = 0; r < s->nrep; ++r) {
        RepParams P = rep_params(s->cfg[r], s->radii[r].data(), t.skin_frac, t.cell);
        P.p_begin = p;
        P.blk_begin = p / kTile;
        P.key_off = key;
        key += P.nkeys;
        p += P.n_pad;
        out.push_back(P);
    }
    *keys = key;
    return out;
}

// Makes t the handle's parameter set (tables on the device; the lists are rebuilt by
// the caller before the next evaluation).
void apply_tune(sim* s, const Tune& t) {
    uint32_t keys = 0;
    s->P = layout(s, t, &keys);
    if (keys > s->keys_cap) throw std::string(fmt("%u cell keys exceed the %u allocated", keys, s->keys_cap));
    s->b.nkeys_total = keys;
    HIPCHK(hipMemcpyAsync(s->b.reps, s->P.data(), sizeof(RepParams) * s->nrep, hipMemcpyHostToDevice, s->st));
    set_variant(s, t.lanes, t.occ);
    s->tune = t;
}

// whether a parameter set keeps every replica's minimum image unique
bool tune_fits(const sim* s, const Tune& t) {
    for (int r = 0; r < s->nrep; ++r)
        if (!box_fits(s->cfg[r], s->radii[r].data(), eff_skin(s->cfg[r], s->radii[r].data(), t.skin_frac)))
            return false;
    return true;
}

// ---- cache of tuned parameter sets: a JSON object, one entry per line,
// "key": {"lanes": L, "occ": O, "skin": F, "cell": C}
std::string g_tune_cache;  // path; empty = no cache (guarded by g_mu)

std::string tune_key(const sim* s) {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) == hipSuccess) (void)hipGetDeviceProperties(&prop, dev);
    const sim_config& c0 = s->cfg[0];
    double ntot = 0.0, phi = 0.0, poly = 1.0, pe = 0.0;
    for (int r = 0; r < s->nrep; ++r) {
        const sim_config& c = s->cfg[r];
        const double* a = s->radii[r].data();
        double v = 0.0;
        for (uint32_t i = 0; i < c.n; ++i) v += (4.0 / 3.0) * kPi * a[i] * a[i] * a[i];
        phi += v / (c.box[0] * c.box[1] * c.box[2]) / s->nrep;
        ntot += c.n;
        poly = std::max(poly, max_radius(a, c.n) / min_radius(a, c.n));
        const double am = min_radius(a, c.n);
        const double p = c.kT > 0.0 ? 6.0 * kPi * c.eta * am * am * am * std::fabs(c.gammadot) / c.kT : 1e30;
        pe += std::log10(std::max(p, 1e-30)) / s->nrep;
    }
    return fmt("%s/%d|%s|flags%x|rep%d|nrep%d|log2n%.1f|phi%.2f|poly%.1f|log10pe%.0f|skin%g|cell%g|lanes%u|kern%u",
               prop.gcnArchName, prop.multiProcessorCount, s->mixed ? "mixed" : "fp64", s->flags,
               c0.repulsion > 0.0 ? 1 : 0, std::min(s->nrep, 64), std::round(2.0 * std::log2(ntot)) / 2.0,
               std::round(phi * 50.0) / 50.0, std::round(poly * 10.0) / 10.0, std::min(pe, 12.0),
               c0.skin < 0.0 ? -1.0 : c0.skin, c0.cell_factor < 0.0 ? -1.0 : c0.cell_factor, c0.lanes,
               c0.pair_kernel);
}

std::vector<std::pair<std::string, Tune>> cache_read(const std::string& path) {
    std::vector<std::pair<std::string, Tune>> out;
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return out;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        const char* q0 = std::strchr(line, '"');
        const char* q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
        const char* br = q1 ? std::strchr(q1, '{') : nullptr;
        if (!br) continue;
        Tune t;
        if (std::sscanf(br, "{\"lanes\": %d, \"occ\": %d, \"skin\": %lf, \"cell\": %lf}", &t.lanes, &t.occ,
                        &t.skin_frac, &t.cell) == 4)
            out.push_back({std::string(q0 + 1, q1), t});
    }
    std::fclose(f);
    return out;
}

void cache_write(const std::string& path, const std::string& key, const Tune& t) {
    auto all = cache_read(path);
    bool found = false;
    for (auto& e : all)
        if (e.first == key) { e.second = t; found = true; }
    if (!found) all.push_back({key, t});
    const std::string tmp = path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;  // a cache that cannot be written is not an error
    std::fprintf(f, "{\n");
    for (size_t k = 0; k < all.size(); ++k)
        std::fprintf(f, "\"%s\": {\"lanes\": %d, \"occ\": %d, \"skin\": %.17g, \"cell\": %.17g}%s\n",
                     all[k].first.c_str(), all[k].second.lanes, all[k].second.occ, all[k].second.skin_frac,
                     all[k].second.cell, k + 1 < all.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    (void)std::rename(tmp.c_str(), path.c_str());
}

// One measured trial of a parameter set on the actual system: rebuild, 2 warm-up
// steps, rebuild (timed), then kRuns runs of kTrial steps (the fastest counts: a run
// can catch a stall).  Returns the expected time per step including the
// rebuilds, from the growth of the displacement bound over the trial (the rule the
// step planner uses): +inf when a list expired during the trial.  The trial steps
// change the state; the caller restores it.
constexpr int kTrial = 8, kRuns = 3;   // steps per timed run of a trial, timed runs

double trial(sim* s, const Tune& t, hipEvent_t* e) {
    apply_tune(s, t);
    const int q = 1 - s->par;
    rebuild(s, q, 0, 0xFFFFFFFFu);
    enqueue_steps(s, s->st, 2, q);
    HIPCHK(hipEventRecord(e[0], s->st));
    rebuild(s, q, 0, 0xFFFFFFFFu);
    HIPCHK(hipEventRecord(e[1], s->st));
    for (int k = 0; k < kRuns; ++k) {
        enqueue_steps(s, s->st, kTrial, q ^ ((k * kTrial) & 1));
        HIPCHK(hipEventRecord(e[2 + k], s->st));
    }
    HIPCHK(hipEventSynchronize(e[1 + kRuns]));
    float mr = 0.f, mbest = 1e30f;
    HIPCHK(hipEventElapsedTime(&mr, e[0], e[1]));
    for (int k = 0; k < kRuns; ++k) {
        float m = 0.f;
        HIPCHK(hipEventElapsedTime(&m, e[1 + k], e[2 + k]));
        mbest = std::min(mbest, m);
    }
    SysDyn sy;
    HIPCHK(hipMemcpy(&sy, s->b.sys, sizeof sy, hipMemcpyDeviceToHost));
    if (sy.halted) return 1e30;
    // fraction of the skin used per step (largest over replicas) over the timed steps
    const int last = q ^ ((kRuns * kTrial - 1) & 1);
    const uint32_t nt = s->b.npad / kTile;
    std::vector<float> dp(nt);
    std::vector<RepDyn> dyn(s->nrep);
    HIPCHK(hipMemcpy(dp.data(), s->b.dpart + (size_t)last * nt, nt * sizeof(float), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(dyn.data(), s->b.dyn, sizeof(RepDyn) * s->nrep, hipMemcpyDeviceToHost));
    double used = 0.0;
    for (int r = 0; r < s->nrep; ++r) {
        const RepParams& P = s->P[r];
        double dmax = 0.0;
        for (uint32_t k = P.blk_begin; k < P.blk_begin + P.nblk; ++k) dmax = std::max(dmax, (double)dp[k]);
        const double u = 2.0 * dmax + std::fabs(P.gd) * dyn[r].t_slot[last] * (P.rc_max + 2.0 * P.skin);
        used = std::max(used, u / P.skin / (double)(kRuns * kTrial));
    }
    const double steps_per_build = used > 0.0 ? std::max(1.0, 0.8 / used) : 1e30;
    return mbest / kTrial + mr / steps_per_build;
}

// Time of one list build under t, the fastest of three from the same positions: the cell
// factor changes nothing but the build (and the analysis passes), so it is chosen by this.
double build_time(sim* s, const Tune& t, hipEvent_t* e) {
    apply_tune(s, t);
    const int q = 1 - s->par;
    rebuild(s, q, 0, 0xFFFFFFFFu);   // regrows the lists if these cells find more partners
    float best = 1e30f;
    for (int k = 0; k < 3; ++k) {
        HIPCHK(hipEventRecord(e[0], s->st));
        launch_rebuild(s->b, s->st, q, 0, 0xFFFFFFFFu);   // the same positions: the same lists
        HIPCHK(hipEventRecord(e[1], s->st));
        HIPCHK(hipEventSynchronize(e[1]));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e[0], e[1]));
        best = std::min(best, ms);
    }
    return best;
}

// Chooses the parameter set: what the configuration fixes is kept; the rest is read
// from the cache or measured on the actual system, one parameter at a time: lanes and
// kernel form, then the skin, by trial(); then the cell factor, by build_time().
void tune(sim* s) {
    const sim_config& c0 = s->cfg[0];
    const bool occ_ok = !s->mixed && !s->b.ext && !(s->flags & SIM_HALF_OCC_OFF);
    std::vector<std::pair<int, int>> forms;  // (lanes, occ)
    for (int L : {1, 2, 4}) {
        if (c0.lanes && (int)c0.lanes != L) continue;
        if (!(occ_ok && (s->flags & SIM_HALF_OCC_ON))) forms.push_back({L, 0});
        if (occ_ok) forms.push_back({L, 1});
    }
    std::vector<double> skins, cells;
    if (c0.skin < 0.0) skins.assign(std::begin(kSkinFracs), std::end(kSkinFracs));
    else skins.push_back(kSkinDefault);
    if (c0.cell_factor < 0.0) cells.assign(std::begin(kCellFactors), std::end(kCellFactors));
    else cells.push_back(1.0);
    Tune best;
    best.lanes = forms[0].first;
    best.occ = forms[0].second;
    best.skin_frac = skins.size() == 1 ? skins[0] : kSkinDefault;
    best.cell = 1.0;
    if (forms.size() == 1 && skins.size() == 1 && cells.size() == 1) {
        apply_tune(s, best);
        return;
    }
    std::string path;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        path = g_tune_cache;
    }
    const std::string key = path.empty() ? std::string() : tune_key(s);
    if (!path.empty()) {
        for (auto& e : cache_read(path)) {
            Tune t = e.second;
            if (e.first != key || !tune_fits(s, t)) continue;
            t.source = 2;
            apply_tune(s, t);
            return;
        }
    }
    hipEvent_t ev[kRuns + 2];
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    auto scan = [&](std::vector<Tune> cand) {
        double bt = 1e31;
        for (const Tune& t : cand) {
            if (!tune_fits(s, t)) continue;
            const double ms = trial(s, t, ev);
            if (ms < bt) { bt = ms; best = t; }
        }
    };
    std::vector<Tune> cand;
    for (auto f : forms) { Tune t = best; t.lanes = f.first; t.occ = f.second; cand.push_back(t); }
    if (cand.size() > 1) scan(cand);
    cand.clear();
    for (double sf : skins) { Tune t = best; t.skin_frac = sf; cand.push_back(t); }
    if (cand.size() > 1) scan(cand);
    if (cells.size() > 1) {
        double bt = 1e31;
        Tune pick = best;
        for (double cf : cells) {
            Tune t = best;
            t.cell = cf;
            if (!tune_fits(s, t)) continue;
            const double ms = build_time(s, t, ev);
            if (ms < bt) { bt = ms; pick = t; }
        }
        best = pick;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    best.source = 1;
    apply_tune(s, best);
    if (!path.empty()) cache_write(path, key, best);
}

int check_rep(sim* s, int32_t r) {
    if (!s) return fail(nullptr, SIM_EINVAL, "null handle");
    if (r < 0 || r >= s->nrep) return fail(s, SIM_ERANGE, fmt("replica %d out of range [0, %d)", r, s->nrep));
    return SIM_OK;
}

}  // namespace

extern "C" {

int sim_validate(const sim_config* cfg, const double* radii) {
    std::string why;
    const int rc = validate(cfg, radii, why);
    if (rc != SIM_OK) set_global_error(why);
    return rc;
}

int sim_set_allocator(void* (*alloc_fn)(size_t, void*), void (*free_fn)(void*, void*), void* ctx) {
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) return fail(nullptr, SIM_EINVAL, "give both or neither");
    std::lock_guard<std::mutex> lk(g_mu);
    g_alloc = alloc_fn;
    g_free = free_fn;
    g_alloc_ctx = ctx;
    return SIM_OK;
}

int sim_set_tune_cache(const char* path) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tune_cache = path ? path : "";
    return SIM_OK;
}

// index of the first NaN or infinity among n values (-1: none, or no array)
static int64_t first_nonfinite(const double* a, uint64_t n) {
    if (!a) return -1;
    for (uint64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return (int64_t)i;
    return -1;
}

int sim_create(const sim_config* cfgs, int32_t n_replicas, const double* const* radii, const double* const* x0,
               const double* const* v0, const double* const* w0, void* hip_stream, sim** out) {
    if (!out) return fail(nullptr, SIM_EINVAL, "null output handle");
    *out = nullptr;
    if (!cfgs || n_replicas <= 0 || !radii || !x0) return fail(nullptr, SIM_EINVAL, "missing replicas");
    for (int r = 0; r < n_replicas; ++r) {
        std::string why;
        if (validate(&cfgs[r], radii[r], why) != SIM_OK) return fail(nullptr, SIM_EINVAL, fmt("replica %d: %s", r, why.c_str()));
        if (cfgs[r].precision != cfgs[0].precision || cfgs[r].flags != cfgs[0].flags ||
            cfgs[r].lanes != cfgs[0].lanes || cfgs[r].pair_kernel != cfgs[0].pair_kernel ||
            (cfgs[r].skin < 0.0) != (cfgs[0].skin < 0.0) || (cfgs[r].cell_factor < 0.0) != (cfgs[0].cell_factor < 0.0))
            return fail(nullptr, SIM_EINVAL, "precision, flags, lanes, pair_kernel and which of skin and cell_factor "
                                             "are tuned must be equal for all replicas");
        if (!x0[r]) return fail(nullptr, SIM_EINVAL, fmt("replica %d: null positions", r));
        for (uint32_t i = 0; i < 3 * cfgs[r].n; ++i) {
            const double L = cfgs[r].box[i % 3];
            if (!(x0[r][i] >= 0.0 && x0[r][i] < L))
                return fail(nullptr, SIM_EINVAL, fmt("replica %d: coordinate %u outside [0, L)", r, i));
        }
        const int64_t bv = first_nonfinite(v0 ? v0[r] : nullptr, 3ull * cfgs[r].n);
        const int64_t bw = first_nonfinite(w0 ? w0[r] : nullptr, 3ull * cfgs[r].n);
        if (bv >= 0 || bw >= 0)
            return fail(nullptr, SIM_EINVAL, fmt("replica %d: %s value %lld is not finite", r, bv >= 0 ? "velocity" :
                                                 "angular velocity", (long long)(bv >= 0 ? bv : bw)));
    }
    sim* s = new sim();
    try {
        {
            std::lock_guard<std::mutex> lk(g_mu);
            s->afn = g_alloc;
            s->ffn = g_free;
            s->actx = g_alloc_ctx;
        }
        s->st = (hipStream_t)hip_stream;
        HIPCHK(hipStreamCreateWithFlags(&s->cap_st, hipStreamNonBlocking));
        s->nrep = n_replicas;
        s->mixed = cfgs[0].precision == SIM_MIXED;
        s->flags = cfgs[0].flags;
        s->cfg.assign(cfgs, cfgs + n_replicas);
        s->ring_tail.assign(n_replicas, 0);
        s->dyn_host.resize(n_replicas);
        uint32_t cap = cfgs[0].nlist_cap ? cfgs[0].nlist_cap : kDefaultCap;
        for (int r = 1; r < n_replicas; ++r) cap = std::max(cap, cfgs[r].nlist_cap ? cfgs[r].nlist_cap : kDefaultCap);
        for (int r = 0; r < n_replicas; ++r) s->radii.emplace_back(radii[r], radii[r] + cfgs[r].n);
        // cell keys for the finest layout any parameter set can ask for (the smallest skin, cells
        // of one list range)
        uint32_t key = 0;
        {
            Tune t;
            t.skin_frac = cfgs[0].skin < 0.0 ? kSkinFracs[0] : kSkinDefault;
            s->P = layout(s, t, &key);
            s->keys_cap = key;
        }
        uint32_t p = 0;
        std::vector<uint32_t> blk_rep;
        for (int r = 0; r < n_replicas; ++r) {
            const sim_config& c = cfgs[r];
            const RepParams& P = s->P[r];
            for (uint32_t k = 0; k < P.nblk; ++k) blk_rep.push_back((uint32_t)r);
            p += P.n_pad;
            double sa3 = 0.0;
            for (uint32_t i = 0; i < c.n; ++i) sa3 += radii[r][i] * radii[r][i] * radii[r][i];
            // Sec. II.B: per-particle drag stresslet 20/3 pi eta a^3 E, E_xy = gammadot / 2 (a
            // stress of the one-body drag: none when that is switched off)
            const double on = (c.flags & SIM_NO_ONEBODY) ? 0.0 : 1.0;
            s->drag_xy.push_back(on * P.invV * (20.0 / 3.0) * kPi * c.eta * sa3 * 0.5 * c.gammadot);
        }
        Bufs& b = s->b;
        b.npad = p;
        b.nrep = (uint32_t)n_replicas;
        b.nkeys_total = key;
        b.cap = cap;
        b.mixed = s->mixed;
        const size_t np = p;
        // list entry slots e * npad + i are 32-bit indices on the device
        if ((uint64_t)np * cap >= (1ull << 32)) throw std::string(fmt("%zu particle slots x %u list entries exceed 2^32", np, cap));
        b.pos = s->alloc<double4>(np);
        b.vh = s->alloc<double4>(np);
        b.wh = s->alloc<double4>(np);
        b.vf = s->alloc<double4>(np);
        b.wf = s->alloc<double4>(np);
        b.F = s->dalloc(np * (s->mixed ? sizeof(float4) : sizeof(double4)));
        b.T = s->dalloc(np * (s->mixed ? sizeof(float4) : sizeof(double4)));
        b.vsh = s->mixed ? s->alloc<float4>(np) : nullptr;
        b.wsh = s->mixed ? s->alloc<float4>(np) : nullptr;
        b.id = s->alloc<uint32_t>(np);
        b.nbr = s->alloc<uint32_t>(np * cap);
        b.ncnt = s->alloc<uint32_t>(np);
        b.hs = s->dalloc(np * cap * 3 * (s->mixed ? sizeof(float) : sizeof(double)));
        b.cmask = s->alloc<uint64_t>(np);
        b.smask = s->alloc<uint64_t>(np);
        b.pidx = s->alloc<PairIdx>(np);
        b.mir = s->alloc<uint8_t>(np * cap);
        b.pf = s->dalloc(np * cap * (s->mixed ? 4 * sizeof(float) : 3 * sizeof(double)));
        b.pt = s->dalloc(np * cap * (s->mixed ? 4 * sizeof(float) : 3 * sizeof(double)));
        b.pt2 = s->dalloc(np * cap * (s->mixed ? 4 * sizeof(float) : 3 * sizeof(double)));
        b.qcap = (s->flags & SIM_SMALL_QUEUE) ? 64u : 2048u;
        b.acf_comp = -1;   // no streaming autocorrelation until asked for
        b.acf_nlag = 0;
        b.rot = (s->flags & SIM_LUB_ROT) ? 1 : 0;
        b.ext = b.rot;
        for (int r = 0; r < n_replicas; ++r)
            if (cfgs[r].repulsion > 0.0) b.ext = 1;
        b.key = s->alloc<uint32_t>(np);
        b.cell_cnt = s->alloc<uint32_t>(key);
        b.cell_fill = s->alloc<uint32_t>(key);
        b.cell_start = s->alloc<uint32_t>(key + 1);
        b.scan_blk = s->alloc<uint32_t>((key + 1023) / 1024 + 1);
        b.src = s->alloc<uint32_t>(np);
        b.ct_id = s->alloc<uint32_t>(np * 2 * kCtCap);
        b.ct_s = s->alloc<double>(np * 2 * kCtCap * 3);
        b.ct_sl = s->alloc<uint8_t>(np * kCtCap);
        b.ct_n = s->alloc<uint32_t>(np * 2);
        for (int a = 0; a < 8; ++a) b.alt4[a] = s->alloc<double4>(np);
        b.disp = s->alloc<double4>(np);
        b.alt_id = s->alloc<uint32_t>(np);
        b.nblk_max = (uint32_t)(np / 256 * 4);               // 256-thread pair blocks, up to 4 lanes
        b.partial = s->alloc<double>((size_t)2 * b.nblk_max * 27);
        b.ovpart = s->alloc<float>((size_t)2 * b.nblk_max);
        b.ring = s->alloc<double>((size_t)n_replicas * kRing * 27);
        b.last = s->alloc<double>((size_t)n_replicas * 27);
        b.blk_rep = s->alloc<uint32_t>(blk_rep.size());
        b.dacc = s->alloc<float>(np);
        b.dpart = s->alloc<float>(2 * (np / kTile));
        b.reps = s->alloc<RepParams>(n_replicas);
        b.dyn = s->alloc<RepDyn>(n_replicas);
        b.sys = s->alloc<SysDyn>(1);
        HIPCHK(hipMemcpyAsync(b.blk_rep, blk_rep.data(), blk_rep.size() * 4, hipMemcpyHostToDevice, s->st));
        HIPCHK(hipMemcpyAsync(b.reps, s->P.data(), sizeof(RepParams) * n_replicas, hipMemcpyHostToDevice, s->st));
        auto load_initial = [&]() {
            for (int r = 0; r < n_replicas; ++r) {
                upload_state(s, r, x0[r], v0 ? v0[r] : nullptr, w0 ? w0[r] : nullptr, nullptr, nullptr, nullptr,
                             nullptr, 0);
                set_dyn(s, r, cfgs[r].le_offset0, cfgs[r].step0);
            }
            HIPCHK(hipMemsetAsync(b.sys, 0, sizeof(SysDyn), s->st));
            HIPCHK(hipMemsetAsync(b.dacc, 0, sizeof(float) * b.npad, s->st));
            s->step_now = cfgs[0].step0;
            rebuild(s, 1 - s->par, 0, 0xFFFFFFFEu);
        };
        {
            Tune t0;
            t0.lanes = cfgs[0].lanes ? (int)cfgs[0].lanes : 1;
            t0.occ = 0;
            t0.skin_frac = kSkinDefault;
            if (cfgs[0].skin < 0.0) t0.skin_frac = kSkinFracs[0];
            apply_tune(s, t0);
        }
        load_initial();
        launch_pair_force(b, s->st, s->par, 0, 0, 0xFFFFFFFFu);
        tune(s);
        // the trial steps moved the state: start again from the initial one
        load_initial();
        launch_pair_force(b, s->st, s->par, 0, 0, 0xFFFFFFFFu);
        launch_finalize(b, s->st, s->par);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s->st));
        const int hc = check_health(s);
        if (hc != SIM_OK) {
            std::string m = s->err;
            delete s;
            return fail(nullptr, hc, m);
        }
    } catch (const HipError& e) {
        std::string m = fmt("%s failed: %s", e.what, hipGetErrorString(e.e));
        delete s;
        return fail(nullptr, e.e == hipErrorOutOfMemory ? SIM_ENOMEM : SIM_EDEVICE, m);
    } catch (const std::string& m) {
        delete s;
        return fail(nullptr, SIM_EINVAL, m);
    }
    *out = s;
    return SIM_OK;
}

namespace {

// Launches m steps on the library stream (chained step graphs, see below,
// or direct launches), then waits.  Step k of the chunk has parity par^1^(k&1).
void launch_steps(sim* s, int64_t m) {
    int q = 1 - s->par;
    const bool graph = !(s->flags & SIM_NO_GRAPH) && !s->profile;
    if (graph) {
        // the m steps form one launch sequence: graphs of kGraphLong steps, then of
        // kGraphSteps, then of 1, chained through the fused gather; only the first
        // integrates, only the last leaves full-step values
        for (bool first = true; m > 0; first = false) {
            const int n = m >= kGraphLong ? kGraphLong : m >= kGraphSteps ? kGraphSteps : 1;
            const bool more = m > n;
            hipGraphExec_t& g = s->gc[n == 1 ? 0 : n == kGraphSteps ? 1 : 2][q][first ? 1 : 0][more ? 1 : 0];
            if (!g) g = capture(s, n, q, first, more);
            HIPCHK(hipGraphLaunch(g, s->st));
            m -= n;
            q ^= n & 1;
        }
    } else if (s->profile) {
        // Kernel times from events the hardware records at each kernel's start and end,
        // on the same launch sequence as the graphs (fused steps, no host wait inside a
        // batch); a batch in which a list expiry halted a step is not counted.
        constexpr int kBatch = 32;
        while (s->ev.size() < 6 * (size_t)kBatch) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            s->ev.push_back(e);
        }
        const bool half = true;  // the gathers integrate every step of a batch but the first
        while (m > 0) {
            const int nb = (int)std::min<int64_t>(m, kBatch);
            for (int k = 0; k < nb; ++k) {
                const int qk = q ^ (k & 1);
                hipEvent_t* e = &s->ev[6 * (size_t)k];
                if (k == 0 || !half) {
                    HIPCHK(hipEventRecord(e[0], s->st));
                    launch_integrate(s->b, s->st, qk);
                    HIPCHK(hipEventRecord(e[1], s->st));
                }
                launch_pair_force(s->b, s->st, qk, 1, 1, 0xFFFFFFFFu, &e[2], half && k + 1 < nb);
            }
            HIPCHK(hipStreamSynchronize(s->st));
            SysDyn sy;
            HIPCHK(hipMemcpy(&sy, s->b.sys, sizeof sy, hipMemcpyDeviceToHost));
            if (sy.halted) break;  // the caller completes the halted step
            for (int k = 0; k < nb; ++k) {
                hipEvent_t* e = &s->ev[6 * (size_t)k];
                float mi = 0.f, mp = 0.f, mg = 0.f;
                if (k == 0 || !half) HIPCHK(hipEventElapsedTime(&mi, e[0], e[1]));
                HIPCHK(hipEventElapsedTime(&mp, e[2], e[3]));
                if (half) HIPCHK(hipEventElapsedTime(&mg, e[4], e[5]));
                s->prof_ms += mp + mg;
                s->prof_stage_ms[0] += mi;
                s->prof_stage_ms[1] += mp;
                s->prof_stage_ms[2] += mg;
                s->prof_launches += 1;
            }
            m -= nb;
            q ^= nb & 1;
        }
    } else {
        enqueue_steps(s, s->st, (int)m, q);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->st));
}

// Steps affordable before the displacement bound can use up the skin, from its
// growth since the last build (the bound grows at most linearly per step).
int64_t plan_steps(sim* s, const std::vector<RepDyn>& dyn) {
    if (s->since_build <= 0) return s->plan_hint;
    // largest displacement bound per replica after the last step's drift (block maxima)
    const uint32_t nt = s->b.npad / kTile;
    std::vector<float> dp(nt);
    HIPCHK(hipMemcpyAsync(dp.data(), s->b.dpart + (size_t)s->par * nt, nt * sizeof(float), hipMemcpyDeviceToHost,
                          s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    double worst = 0.0;  // fraction of the skin used per step
    for (int r = 0; r < s->nrep; ++r) {
        const RepParams& P = s->P[r];
        double dmax = 0.0;
        for (uint32_t k = P.blk_begin; k < P.blk_begin + P.nblk; ++k) dmax = std::max(dmax, (double)dp[k]);
        const double used = 2.0 * dmax + std::fabs(P.gd) * dyn[r].t_slot[s->par] * (P.rc_max + 2.0 * P.skin);
        worst = std::max(worst, used / P.skin / (double)s->since_build);
    }
    if (!(worst > 0.0)) return 1 << 20;
    return (int64_t)(0.8 / worst);
}

}  // namespace

int sim_step(sim* s, int64_t nsteps) {
    if (!s) return fail(nullptr, SIM_EINVAL, "null handle");
    if (nsteps < 0) return fail(s, SIM_EINVAL, "nsteps < 0");
    try {
        ensure_lists(s);
        int64_t left = nsteps;
        std::vector<RepDyn> dyn(s->nrep);
        const bool every = (s->flags & SIM_REBUILD_EACH_STEP) != 0;
        while (left > 0) {
            int64_t budget = every ? 0 : s->plan - s->since_build;
            if (budget < 1) {
                // displacement budget used up: rebuild between steps, from the current positions
                rebuild(s, 1 - s->par, 0, 0xFFFFFFFFu);
                s->since_build = 0;
                s->plan = s->plan_hint;
                budget = every ? 1 : s->plan;
            }
            const int64_t m = std::min(left, std::max<int64_t>(budget, 1));
            launch_steps(s, m);
            HIPCHK(hipMemcpyAsync(dyn.data(), s->b.dyn, sizeof(RepDyn) * s->nrep, hipMemcpyDeviceToHost, s->st));
            SysDyn sy;
            HIPCHK(hipMemcpyAsync(&sy, s->b.sys, sizeof sy, hipMemcpyDeviceToHost, s->st));
            HIPCHK(hipStreamSynchronize(s->st));
            const uint64_t cur = std::max(dyn[0].step_slot[0], dyn[0].step_slot[1]);
            const int64_t done = (int64_t)(cur - s->step_now);
            s->step_now = cur;
            s->par ^= (int)(done & 1);
            s->since_build += done;
            left -= done;
            if (sy.halted) {
                // the next step ran its integrate but the expiry test stopped its forces:
                // rebuild from the moved positions and evaluate that step
                const int64_t grown = plan_steps(s, dyn);
                const int q = 1 - s->par;
                rebuild(s, q, 1, 0xFFFFFFFFu);
                launch_pair_force(s->b, s->st, q, 1, 1, 0xFFFFFFFFu);
                HIPCHK(hipGetLastError());
                HIPCHK(hipStreamSynchronize(s->st));
                s->par = q;
                s->step_now += 1;
                left -= 1;
                s->plan_hint = std::max<int64_t>(1, std::min<int64_t>(grown, s->since_build + 1) / 2);
                s->since_build = 0;
                s->plan = s->plan_hint;
            } else {
                const int64_t p = plan_steps(s, dyn);
                s->plan = std::max<int64_t>(s->since_build + 1, std::min<int64_t>(p, 1 << 20));
                if (p <= s->since_build) s->plan = s->since_build;  // rebuild before the next chunk
                s->plan_hint = std::max<int64_t>(16, std::min<int64_t>(p, 1 << 20));
            }
        }
        // reduce the stress of the last step (earlier steps were reduced by the next integrate)
        launch_finalize(s->b, s->st, s->par);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s->st));
        s->steps_total += nsteps;
        return check_health(s);
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_profile(sim* s, int32_t enable) {
    if (!s) return fail(nullptr, SIM_EINVAL, "null handle");
    s->profile = enable ? 1 : 0;
    s->prof_launches = 0;
    s->prof_ms = 0.0;
    for (double& t : s->prof_stage_ms) t = 0.0;
    return SIM_OK;
}

int sim_stage_time(sim* s, int32_t stage, int64_t* launches, double* total_ms) {
    if (!s) return fail(nullptr, SIM_EINVAL, "null handle");
    if (stage < 0 || stage > 2) return fail(s, SIM_EINVAL, "stage must be 0, 1 or 2");
    if (launches) *launches = s->prof_launches;
    if (total_ms) *total_ms = s->prof_stage_ms[stage];
    return SIM_OK;
}

int sim_kernel_time(sim* s, int64_t* launches, double* total_ms) {
    if (!s) return fail(nullptr, SIM_EINVAL, "null handle");
    if (launches) *launches = s->prof_launches;
    if (total_ms) *total_ms = s->prof_ms;
    return SIM_OK;
}

int sim_stress(sim* s, int32_t r, int32_t component, int32_t mode, double out[9]) {
    if (int rc = check_rep(s, r)) return rc;
    if (!out || component < 0 || component > SIM_STRESS_TOTAL || (mode != SIM_STRESS_LAST && mode != SIM_STRESS_MEAN))
        return fail(s, SIM_EINVAL, "bad component, mode or output");
    try {
        double v[27];
        if (mode == SIM_STRESS_LAST) {
            auto h = d2h(s, s->b.last, (size_t)r * 27, 27);
            std::copy(h.begin(), h.end(), v);
        } else {
            auto d = d2h(s, s->b.dyn, (size_t)r, 1);
            const uint32_t n = d[0].nrec - d[0].rec_base;
            const double c = n ? (double)n : 1.0;
            for (int k = 0; k < 27; ++k) v[k] = d[0].stress_sum[k] / c;
        }
        double drag[9] = {0, s->drag_xy[r], 0, s->drag_xy[r], 0, 0, 0, 0, 0};
        for (int k = 0; k < 9; ++k) {
            switch (component) {
                case SIM_STRESS_CONTACT: out[k] = v[k]; break;
                case SIM_STRESS_LUB: out[k] = v[9 + k]; break;
                case SIM_STRESS_BROWN: out[k] = v[18 + k]; break;
                case SIM_STRESS_DRAG: out[k] = drag[k]; break;
                default: out[k] = v[k] + v[9 + k] + drag[k]; break;
            }
        }
        return SIM_OK;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_reset_stress(sim* s) {
    if (!s) return fail(nullptr, SIM_EINVAL, "null handle");
    try {
        std::vector<RepDyn> dyn(s->nrep);
        HIPCHK(hipMemcpyAsync(dyn.data(), s->b.dyn, sizeof(RepDyn) * s->nrep, hipMemcpyDeviceToHost, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
        const double z[27] = {0};
        if (s->b.acf_hist) {   // the streaming autocorrelation starts again
            launch_zero64(s->st, (unsigned long long*)s->b.acf_sum, (uint32_t)((size_t)s->nrep * s->b.acf_nlag));
            launch_zero64(s->st, s->b.acf_n, (uint32_t)s->nrep);
        }
        for (int r = 0; r < s->nrep; ++r) {
            HIPCHK(hipMemcpyAsync((char*)(s->b.dyn + r) + offsetof(RepDyn, stress_sum), z, sizeof z,
                                  hipMemcpyHostToDevice, s->st));
            HIPCHK(hipMemcpyAsync((char*)(s->b.dyn + r) + offsetof(RepDyn, rec_base), &dyn[r].nrec, sizeof(uint32_t),
                                  hipMemcpyHostToDevice, s->st));
        }
        HIPCHK(hipStreamSynchronize(s->st));
        return SIM_OK;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_stress_series(sim* s, int32_t r, double* out, int64_t cap, int64_t* count) {
    if (int rc = check_rep(s, r)) return rc;
    if (!count) return fail(s, SIM_EINVAL, "null count");
    try {
        auto d = d2h(s, s->b.dyn, (size_t)r, 1);
        const uint32_t head = d[0].nrec;  // records 1..head; record k sits in slot (k - 1) % kRing
        uint32_t tail = s->ring_tail[r];
        if (head - tail > (uint32_t)kRing) tail = head - kRing;
        const int64_t n = (int64_t)(head - tail);
        *count = n;
        if (n > cap || (!out && n > 0)) return fail(s, SIM_ERANGE, fmt("series holds %lld steps", (long long)n));
        auto ring = d2h(s, s->b.ring, (size_t)r * kRing * 27, (size_t)kRing * 27);
        for (int64_t k = 0; k < n; ++k) {
            const uint32_t slot = (tail + (uint32_t)k) % kRing;
            std::memcpy(out + 27 * k, ring.data() + (size_t)slot * 27, 27 * sizeof(double));
        }
        s->ring_tail[r] = head;
        return SIM_OK;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_get_state(sim* s, int32_t r, double* x, double* v, double* w, double* F, double* T, double* le_offset,
                  uint64_t* step) {
    if (int rc = check_rep(s, r)) return rc;
    try {
        const RepParams& P = s->P[r];
        const size_t p0 = P.p_begin, np = P.n_pad;
        auto id = d2h(s, s->b.id, p0, np);
        auto scatter4 = [&](const double4* dev, double* outp) {
            if (!outp) return;
            auto h = d2h(s, dev, p0, np);
            for (size_t q = 0; q < np; ++q) {
                if (id[q] == kNoId) continue;
                outp[3 * id[q]] = h[q].x; outp[3 * id[q] + 1] = h[q].y; outp[3 * id[q] + 2] = h[q].z;
            }
        };
        auto scatterF = [&](void* dev, double* outp) {
            if (!outp) return;
            if (s->mixed) {
                auto h = d2h(s, (const float4*)dev, p0, np);
                for (size_t q = 0; q < np; ++q) {
                    if (id[q] == kNoId) continue;
                    outp[3 * id[q]] = h[q].x; outp[3 * id[q] + 1] = h[q].y; outp[3 * id[q] + 2] = h[q].z;
                }
            } else {
                scatter4((const double4*)dev, outp);
            }
        };
        scatter4(s->b.pos, x);
        scatter4(s->b.vf, v);
        scatter4(s->b.wf, w);
        scatterF(s->b.F, F);
        scatterF(s->b.T, T);
        if (le_offset || step) {
            auto d = d2h(s, s->b.dyn, (size_t)r, 1);
            if (le_offset) *le_offset = d[0].s_slot[s->par];
            if (step) *step = d[0].step_slot[s->par];
        }
        return SIM_OK;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_reset_displacement(sim* s) {
    if (s && !(s->flags & SIM_TRACK_DISPLACEMENT))
        return fail(s, SIM_EINVAL, "displacements are kept only by a handle created with SIM_TRACK_DISPLACEMENT");
    if (!s) return fail(nullptr, SIM_EINVAL, "null handle");
    try {
        HIPCHK(hipMemsetAsync(s->b.disp, 0, sizeof(double4) * s->b.npad, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
        return SIM_OK;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_displacement(sim* s, int32_t r, double* out_3n) {
    if (s && !(s->flags & SIM_TRACK_DISPLACEMENT))
        return fail(s, SIM_EINVAL, "displacements are kept only by a handle created with SIM_TRACK_DISPLACEMENT");
    if (int rc = check_rep(s, r)) return rc;
    if (!out_3n) return fail(s, SIM_EINVAL, "null output");
    try {
        const RepParams& P = s->P[r];
        auto id = d2h(s, s->b.id, P.p_begin, P.n_pad);
        auto d = d2h(s, s->b.disp, P.p_begin, P.n_pad);
        for (size_t q = 0; q < P.n_pad; ++q) {
            if (id[q] == kNoId) continue;
            out_3n[3 * id[q]] = d[q].x;
            out_3n[3 * id[q] + 1] = d[q].y;
            out_3n[3 * id[q] + 2] = d[q].z;
        }
        return SIM_OK;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_msd(sim* s, int32_t r, double out[3]) {
    if (int rc = check_rep(s, r)) return rc;
    if (!(s->flags & SIM_TRACK_DISPLACEMENT))
        return fail(s, SIM_EINVAL, "displacements are kept only by a handle created with SIM_TRACK_DISPLACEMENT");
    if (!out) return fail(s, SIM_EINVAL, "null output");
    try {
        const RepParams& P = s->P[r];
        const uint32_t nblk = P.n_pad / 256;
        if (s->struct_cap < nblk) {
            s->struct_part = s->alloc<double>((size_t)nblk * 9);
            s->struct_cap = nblk;
        }
        launch_msd(s->b, s->st, (uint32_t)r, nblk, s->struct_part);
        HIPCHK(hipGetLastError());
        auto h = d2h(s, s->struct_part, 0, (size_t)nblk * 3);
        double acc[3] = {0, 0, 0};
        for (uint32_t k = 0; k < nblk; ++k)
            for (int c = 0; c < 3; ++c) acc[c] += h[(size_t)k * 3 + c];
        for (int c = 0; c < 3; ++c) out[c] = acc[c] / (double)P.n;
        return SIM_OK;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

namespace {
// Pair histogram of replica r into the device array dc (nwords 64-bit counts, zeroed here
// by a kernel), copied to counts: mode 0 = g(r) bins, mode 1 = the flow-gradient slice.
// grow false: allocates nothing (lists that the build finds short are regrown later).
int rdf_into(sim* s, int32_t r, int mode, double r_max, double slab, int32_t nbins, unsigned long long* dc,
             uint64_t* counts, bool grow = true) {
    const RepParams& P = s->P[r];
    const uint32_t nwords = mode == 0 ? (uint32_t)nbins : (uint32_t)nbins * (uint32_t)nbins;
    const double reach = mode == 0 ? r_max : std::sqrt(2.0 * r_max * r_max + 0.25 * slab * slab);
    rebuild(s, 1 - s->par, 0, 0xFFFFFFFFu, grow);   // current cells (changes no trajectory)
    s->since_build = 0;
    s->plan = s->plan_hint;
    launch_zero64(s->st, dc, nwords);
    launch_rdf(s->b, s->st, s->par, (uint32_t)r, P.n_pad / 256, mode, r_max, slab, reach, (uint32_t)nbins, dc);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(counts, dc, sizeof(uint64_t) * nwords, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return check_health(s);
}

// the minimum image of every pair within reach must be unique
bool reach_ok(const RepParams& P, double reach) {
    return reach > 0.0 && reach < 0.5 * std::min(P.L[0], std::min(P.L[1], P.L[2]));
}
}  // namespace

int sim_rdf(sim* s, int32_t r, double r_max, int32_t nbins, uint64_t* counts) {
    if (int rc = check_rep(s, r)) return rc;
    if (!counts || nbins <= 0 || nbins > (1 << 24)) return fail(s, SIM_EINVAL, "need counts and 0 < nbins <= 2^24");
    if (!reach_ok(s->P[r], r_max)) return fail(s, SIM_EINVAL, "r_max must be in (0, L/2) for the smallest box side L");
    try {
        unsigned long long* dc = s->alloc<unsigned long long>((size_t)nbins);
        const int rc = rdf_into(s, r, 0, r_max, 0.0, nbins, dc, counts);
        s->release(dc);
        return rc;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_rdf_noalloc(sim* s, int32_t r, double r_max, int32_t nbins, uint64_t* counts) {
    if (int rc = check_rep(s, r)) return rc;
    if (!counts || nbins <= 0 || nbins > (int32_t)kScratchWords)
        return fail(s, SIM_EINVAL, fmt("need counts and 0 < nbins <= %u (the static scratch array)", kScratchWords));
    if (!reach_ok(s->P[r], r_max)) return fail(s, SIM_EINVAL, "r_max must be in (0, L/2) for the smallest box side L");
    std::string err;
    unsigned long long* dc = scratch_ptr(err);
    if (!dc) return fail(s, SIM_EDEVICE, err);
    try {
        return rdf_into(s, r, 0, r_max, 0.0, nbins, dc, counts, false);
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_rdf_xy(sim* s, int32_t r, double r_max, double slab, int32_t nbins, uint64_t* counts) {
    if (int rc = check_rep(s, r)) return rc;
    if (!counts || nbins <= 0 || nbins > 4096) return fail(s, SIM_EINVAL, "need counts and 0 < nbins <= 4096");
    if (!(slab > 0.0) || !reach_ok(s->P[r], std::sqrt(2.0 * r_max * r_max + 0.25 * slab * slab)))
        return fail(s, SIM_EINVAL, "need slab > 0, r_max > 0 and sqrt(2 r_max^2 + slab^2 / 4) < L/2");
    try {
        unsigned long long* dc = s->alloc<unsigned long long>((size_t)nbins * (size_t)nbins);
        const int rc = rdf_into(s, r, 1, r_max, slab, nbins, dc, counts);
        s->release(dc);
        return rc;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_stress_acf_stream(sim* s, int32_t component, int32_t alpha, int32_t beta, int64_t nlag) {
    if (!s) return fail(nullptr, SIM_EINVAL, "null handle");
    if (nlag < 0 || nlag > (1 << 20)) return fail(s, SIM_EINVAL, "nlag must be in [0, 2^20]");
    if (nlag > 0 && (component < 0 || component > SIM_STRESS_BROWN || alpha < 0 || alpha > 2 || beta < 0 || beta > 2))
        return fail(s, SIM_EINVAL, "bad component or index");
    try {
        HIPCHK(hipStreamSynchronize(s->st));
        if (s->b.acf_hist) {
            s->release(s->b.acf_hist);
            s->release(s->b.acf_sum);
            s->release(s->b.acf_n);
            s->b.acf_hist = s->b.acf_sum = nullptr;
            s->b.acf_n = nullptr;
        }
        s->b.acf_comp = -1;
        s->b.acf_nlag = 0;
        if (nlag > 0) {
            s->b.acf_hist = s->alloc<double>((size_t)s->nrep * nlag);   // zeroed
            s->b.acf_sum = s->alloc<double>((size_t)s->nrep * nlag);
            s->b.acf_n = s->alloc<unsigned long long>((size_t)s->nrep);
            s->b.acf_comp = component * 9 + alpha * 3 + beta;
            s->b.acf_nlag = (uint32_t)nlag;
        }
        drop_graphs(s);   // captured launches hold the buffer table by value
        HIPCHK(hipStreamSynchronize(s->st));
        return SIM_OK;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_stress_acf(sim* s, int32_t r, int32_t component, int32_t alpha, int32_t beta, int64_t nlag, double* out) {
    if (int rc = check_rep(s, r)) return rc;
    if (!out || component < 0 || component > SIM_STRESS_BROWN || alpha < 0 || alpha > 2 || beta < 0 || beta > 2 ||
        nlag <= 0)
        return fail(s, SIM_EINVAL, "bad component, index, lag count or output");
    try {
        const int comp = component * 9 + alpha * 3 + beta;
        if (comp == s->b.acf_comp && nlag <= (int64_t)s->b.acf_nlag) {
            // the streaming sums: every record since the stream started or the stress was reset
            auto n = d2h(s, s->b.acf_n, (size_t)r, 1);
            auto sum = d2h(s, s->b.acf_sum, (size_t)r * s->b.acf_nlag, (size_t)nlag);
            if ((int64_t)n[0] < nlag) return fail(s, SIM_ERANGE, fmt("%llu records streamed, %lld lags asked",
                                                                      (unsigned long long)n[0], (long long)nlag));
            for (int64_t k = 0; k < nlag; ++k) out[k] = sum[k] / (double)(n[0] - (uint64_t)k);
            return SIM_OK;
        }
        auto d = d2h(s, s->b.dyn, (size_t)r, 1);
        const uint32_t head = d[0].nrec;  // records 1..head; record k sits in slot (k - 1) % kRing
        uint32_t first = d[0].rec_base;
        if (head - first > (uint32_t)kRing) first = head - kRing;
        const uint32_t count = head - first;
        if ((int64_t)count < nlag) return fail(s, SIM_ERANGE, fmt("%u records since the reset, %lld lags asked", count, (long long)nlag));
        double* dout = s->alloc<double>((size_t)nlag);
        launch_acf(s->b, s->st, (uint32_t)r, comp, first % kRing, count, (uint32_t)nlag, dout);
        HIPCHK(hipGetLastError());
        auto h = d2h(s, dout, 0, (size_t)nlag);
        std::copy(h.begin(), h.end(), out);
        s->release(dout);
        return SIM_OK;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_structural_stress(sim* s, int32_t r, double out[9]) {
    if (int rc = check_rep(s, r)) return rc;
    if (!out) return fail(s, SIM_EINVAL, "null output");
    const RepParams& P = s->P[r];
    // the list (range (a_i + a_j)(1 + xi_cut/2) + skin) must hold every shell partner
    const double amin = min_radius(s->radii[r].data(), P.n), amax = max_radius(s->radii[r].data(), P.n);
    if (P.skin + amin * (2.0 * (P.c_int - 1.0)) < 0.05 * amax)
        return fail(s, SIM_EINVAL, "the neighbour list range does not cover the 0.05 a shell");
    try {
        rebuild(s, 1 - s->par, 0, 0xFFFFFFFFu);
        s->since_build = 0;
        s->plan = s->plan_hint;
        const uint32_t nblk = P.n_pad / 256;
        if (s->struct_cap < nblk) {
            s->struct_part = s->alloc<double>((size_t)nblk * 9);
            s->struct_cap = nblk;
        }
        launch_struct(s->b, s->st, s->par, (uint32_t)r, nblk, s->struct_part);
        HIPCHK(hipGetLastError());
        auto h = d2h(s, s->struct_part, 0, (size_t)nblk * 9);
        double acc[9] = {0};
        for (uint32_t k = 0; k < nblk; ++k)
            for (int c = 0; c < 9; ++c) acc[c] += h[(size_t)k * 9 + c];
        const double V = P.L[0] * P.L[1] * P.L[2];
        for (int c = 0; c < 9; ++c) out[c] = -P.kT / V * acc[c];
        return check_health(s);
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_positions(sim* s, int32_t r, double* out_3n) {
    if (!out_3n) return fail(s, SIM_EINVAL, "null output");
    return sim_get_state(s, r, out_3n, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
}

int sim_forces(sim* s, int32_t r, double* F_3n, double* T_3n) {
    return sim_get_state(s, r, nullptr, nullptr, nullptr, F_3n, T_3n, nullptr, nullptr);
}

int sim_set_state(sim* s, int32_t r, const double* x, const double* v, const double* w, const double* F,
                  const double* T, double le_offset, uint64_t step, const uint32_t* c_ij, const double* c_s,
                  int64_t n_contacts) {
    if (int rc = check_rep(s, r)) return rc;
    if (!x || !v || !w) return fail(s, SIM_EINVAL, "x, v and w are required");
    if ((F == nullptr) != (T == nullptr)) return fail(s, SIM_EINVAL, "give both F and T or neither");
    if (n_contacts < 0 || (n_contacts > 0 && (!c_ij || !c_s))) return fail(s, SIM_EINVAL, "bad contact arrays");
    const RepParams& P = s->P[r];
    for (uint32_t i = 0; i < 3 * P.n; ++i)
        if (!(x[i] >= 0.0 && x[i] < P.L[i % 3])) return fail(s, SIM_EINVAL, fmt("coordinate %u outside [0, L)", i));
    const char* names[5] = {"velocity", "angular velocity", "force", "torque", "spring"};
    const double* arrays[5] = {v, w, F, T, c_s};
    const uint64_t counts[5] = {3ull * P.n, 3ull * P.n, 3ull * P.n, 3ull * P.n, 3ull * (uint64_t)n_contacts};
    for (int k = 0; k < 5; ++k)
        if (const int64_t b = first_nonfinite(arrays[k], counts[k]); b >= 0)
            return fail(s, SIM_EINVAL, fmt("%s value %lld is not finite", names[k], (long long)b));
    try {
        upload_state(s, r, x, v, w, F, T, c_ij, c_s, n_contacts);
        set_dyn(s, r, le_offset, step);
        if (r == 0) s->step_now = step;
        rebuild(s, 1 - s->par, 0, (uint32_t)r);
        s->since_build = 0;
        if (!F) {
            launch_pair_force(s->b, s->st, s->par, 0, 0, (uint32_t)r);
            launch_finalize(s->b, s->st, s->par);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s->st));
        return check_health(s);
    } catch (const HipError& e) {
        return hip_fail(s, e);
    } catch (const std::string& m) {
        return fail(s, SIM_EINVAL, m);
    }
}

namespace {
// Lists pairs of one replica from the device (mode 0 interaction set, 1
// Verlet list, 2 contacts), sorted by (id_i, id_j).
int diag_pairs(sim* s, int32_t r, int mode, std::vector<uint32_t>& ij, std::vector<double>& sv,
               std::vector<int32_t>& sl) {
    const RepParams& P = s->P[r];
    ensure_lists(s);
    // device buffers through the handle's allocator (the hook, when one is set), freed on every path
    std::vector<void*> held;
    struct Release {
        sim* s;
        std::vector<void*>& p;
        ~Release() {
            for (void* q : p) s->release(q);
        }
    } rel{s, held};
    auto get = [&](size_t bytes) {
        void* q = s->dalloc(bytes);   // zeroed
        held.push_back(q);
        return q;
    };
    uint32_t* dcount = (uint32_t*)get(sizeof(uint32_t));
    launch_diag(s->b, s->st, s->par, (uint32_t)r, P.n, nullptr, nullptr, nullptr, dcount, 0, mode);
    uint32_t cnt = 0;
    HIPCHK(hipMemcpyAsync(&cnt, dcount, 4, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    uint32_t* dij = (uint32_t*)get(sizeof(uint32_t) * 2 * ((size_t)cnt + 1));
    double* ds = (double*)get(sizeof(double) * 3 * ((size_t)cnt + 1));
    int32_t* dsl = (int32_t*)get(sizeof(int32_t) * ((size_t)cnt + 1));
    HIPCHK(hipMemsetAsync(dcount, 0, sizeof(uint32_t), s->st));
    launch_diag(s->b, s->st, s->par, (uint32_t)r, P.n, dij, ds, dsl, dcount, cnt, mode);
    std::vector<uint32_t> hij(2 * (size_t)cnt);
    std::vector<double> hs(3 * (size_t)cnt);
    std::vector<int32_t> hsl(cnt);
    HIPCHK(hipMemcpyAsync(hij.data(), dij, hij.size() * 4, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(hs.data(), ds, hs.size() * 8, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(hsl.data(), dsl, hsl.size() * 4, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    std::vector<uint32_t> order(cnt);
    for (uint32_t k = 0; k < cnt; ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return hij[2 * a] != hij[2 * b] ? hij[2 * a] < hij[2 * b] : hij[2 * a + 1] < hij[2 * b + 1];
    });
    ij.resize(2 * (size_t)cnt);
    sv.resize(3 * (size_t)cnt);
    sl.resize(cnt);
    for (uint32_t k = 0; k < cnt; ++k) {
        const uint32_t o = order[k];
        ij[2 * k] = hij[2 * o];
        ij[2 * k + 1] = hij[2 * o + 1];
        for (int d = 0; d < 3; ++d) sv[3 * k + d] = hs[3 * o + d];
        sl[k] = hsl[o];
    }
    return SIM_OK;
}

int copy_pairs(sim* s, int32_t r, int mode, uint32_t* ij_2m, double* s_3m, int32_t* sliding, int64_t cap,
               int64_t* count) {
    if (int rc = check_rep(s, r)) return rc;
    if (!count) return fail(s, SIM_EINVAL, "null count");
    try {
        std::vector<uint32_t> ij;
        std::vector<double> sv;
        std::vector<int32_t> sl;
        diag_pairs(s, r, mode, ij, sv, sl);
        const int64_t n = (int64_t)sl.size();
        *count = n;
        if (n > cap) return fail(s, SIM_ERANGE, fmt("%lld pairs do not fit in %lld", (long long)n, (long long)cap));
        if (n && !ij_2m) return fail(s, SIM_EINVAL, "null output");
        std::memcpy(ij_2m, ij.data(), ij.size() * 4);
        if (s_3m) std::memcpy(s_3m, sv.data(), sv.size() * 8);
        if (sliding) std::memcpy(sliding, sl.data(), sl.size() * 4);
        return SIM_OK;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}
}  // namespace

int sim_pairs(sim* s, int32_t r, uint32_t* ij_2m, int64_t cap, int64_t* count) {
    return copy_pairs(s, r, 0, ij_2m, nullptr, nullptr, cap, count);
}

int sim_nlist(sim* s, int32_t r, uint32_t* ij_2m, int64_t cap, int64_t* count) {
    return copy_pairs(s, r, 1, ij_2m, nullptr, nullptr, cap, count);
}

int sim_contacts(sim* s, int32_t r, uint32_t* ij_2m, double* s_3m, int32_t* sliding, int64_t cap, int64_t* count) {
    return copy_pairs(s, r, 2, ij_2m, s_3m, sliding, cap, count);
}

int sim_stats(sim* s, int32_t r, sim_stats_t* out) {
    if (int rc = check_rep(s, r)) return rc;
    if (!out) return fail(s, SIM_EINVAL, "null output");
    try {
        std::vector<uint32_t> ij;
        std::vector<double> sv;
        std::vector<int32_t> sl;
        const double n = (double)s->P[r].n;
        diag_pairs(s, r, 2, ij, sv, sl);
        int64_t nsl = 0;
        for (int32_t v : sl) nsl += v;
        out->contacts = (int64_t)sl.size();
        out->contacts_per_particle = 2.0 * (double)sl.size() / n;
        out->sliding_fraction = sl.empty() ? 0.0 : (double)nsl / (double)sl.size();
        diag_pairs(s, r, 1, ij, sv, sl);
        out->neighbours_per_particle = 2.0 * (double)sl.size() / n;
        diag_pairs(s, r, 0, ij, sv, sl);
        out->interacting_per_particle = 2.0 * (double)sl.size() / n;
        auto d = d2h(s, s->b.dyn, (size_t)r, 1);
        auto sy = d2h(s, s->b.sys, 0, 1);
        float mo;
        std::memcpy(&mo, &d[0].maxov_last_bits, sizeof mo);
        out->max_overlap = (double)mo;
        out->rebuilds = (int64_t)sy[0].rebuilds;
        out->steps = s->steps_total;
        out->step = d[0].step_slot[s->par];
        out->le_offset = d[0].s_slot[s->par];
        out->lanes = s->b.lanes;
        out->pair_kernel = SIM_KERNEL_HALF;
        out->occupancy_form = s->b.occ && !s->mixed && !s->b.ext ? 1 : 0;
        out->tune_source = s->tune.source;
        out->skin = s->P[r].skin;
        out->cell_factor = s->cfg[r].cell_factor > 0.0 ? s->cfg[r].cell_factor : s->tune.cell;
        {   // kinetic temperatures of the peculiar motion (fixed-order sums on the device)
            const uint32_t nblk = s->P[r].n_pad / 256;
            if (s->struct_cap < nblk) {
                s->struct_part = s->alloc<double>((size_t)nblk * 9);
                s->struct_cap = nblk;
            }
            launch_kinetic(s->b, s->st, (uint32_t)r, nblk, s->struct_part);
            HIPCHK(hipGetLastError());
            auto h = d2h(s, s->struct_part, 0, (size_t)nblk * 2);
            double ke[2] = {0.0, 0.0};
            for (uint32_t k = 0; k < nblk; ++k)
                for (int c = 0; c < 2; ++c) ke[c] += h[(size_t)k * 2 + c];
            out->kT_translational = ke[0] / (3.0 * n);
            out->kT_rotational = ke[1] / (3.0 * n);
        }
        out->cells_x = s->P[r].nc[0];
        out->cells_y = s->P[r].nc[1];
        out->cells_z = s->P[r].nc[2];
        out->list_cap = (int32_t)s->b.cap;
        return SIM_OK;
    } catch (const HipError& e) {
        return hip_fail(s, e);
    }
}

int sim_destroy(sim* s) {
    delete s;
    return SIM_OK;
}

const char* sim_strerror(int32_t code) {
    switch (code) {
        case SIM_OK: return "ok";
        case SIM_EINVAL: return "invalid configuration or argument";
        case SIM_ENOMEM: return "out of memory";
        case SIM_EDEVICE: return "HIP runtime error";
        case SIM_EUNSTABLE: return "unstable step (non-finite force or overlap above the limit)";
        case SIM_ECAPACITY: return "neighbour list or contact capacity exceeded";
        case SIM_ERANGE: return "index or output capacity out of range";
        default: return "unknown status";
    }
}

int sim_last_error(const sim* s, char* buf, size_t len) {
    if (!buf || len == 0) return SIM_EINVAL;
    std::string m;
    if (s) m = s->err;
    else {
        std::lock_guard<std::mutex> lk(g_mu);
        m = g_err;
    }
    std::snprintf(buf, len, "%s", m.c_str());
    return SIM_OK;
}

}  // extern "C"
