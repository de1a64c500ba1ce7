// Internal declarations of the gfx950 force engine: per-replica parameter
// tables, device buffers and kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace susp {

constexpr int kTile = 256;               // replicas are padded to multiples of this many particles
constexpr uint32_t kNoId = 0xFFFFFFFFu;  // id of a padding slot
constexpr double kPi = 3.14159265358979323846;

enum : uint32_t {
    F_FREEZE_X = 0x001u, F_NO_LUB = 0x002u, F_NO_PAIR_BROWN = 0x004u, F_NO_CONTACT = 0x008u,
    F_NO_ONEBODY = 0x010u, F_LUB_ROT = 0x020u, F_REBUILD_EACH_STEP = 0x100u, F_NO_GRAPH = 0x200u,
    F_TRACK_DISP = 0x2000u,
};

enum : uint32_t { H_NAN = 1u, H_OVERLAP = 2u, H_NLIST = 4u };

// Constant per-replica parameters (host-written, read-only on device).
struct RepParams {
    double L[3];
    double invL[3];
    double gd, gdLy;          // shear rate, shear rate * Ly
    double dt, half_dt;
    double rho, eta, kn, kt, mu;
    double rep_A;             // short-ranged repulsion scale A (0 = none)
    double kT;
    double bamp;              // sqrt(2 kT / dt)
    double c1;                // 1 + xi_cut / 2: lubrication range factor
    double c_int;             // range factor of the pairs evaluated: c1, or with the repulsion
                              // on, max(c1, 1 + 16 * 0.01) (its range of 16 kappa)
    double xi_min;
    double skin;
    double rc_max;            // largest interaction range (2 a_max c_int)
    double rl_max;            // rc_max + skin
    double invV;
    double cw[3];             // cell widths
    double max_overlap;
    int32_t nc[3];            // cells per dimension (1 or >= 3)
    int32_t mbits;            // cell-key bits per dimension (Hilbert order)
    uint32_t key_off;         // first cell key of this replica
    uint32_t nkeys;           // 2^(3 mbits) cell keys + 1 padding cell
    uint32_t p_begin, n, n_pad;
    uint32_t flags;
    uint32_t blk_begin, nblk; // pair-kernel blocks of this replica
    uint64_t seed;
};

// Per-replica values the device updates every step.  Step-dependent values
// are double-buffered by the parity q of the step: a step with parity q reads
// slot 1 - q (the previous step) and writes slot q, so no kernel reads a value
// another block of the same kernel may be writing.
struct RepDyn {
    double s_slot[2];         // Lees-Edwards offset of the evaluation with that parity
    uint64_t step_slot[2];    // step counter of that evaluation
    double t_slot[2];         // time since the last build
    uint32_t eval_id[2];      // serial number of the evaluation whose partials have that parity
    uint32_t rec[2];          // its series record number (1-based), 0 = not recorded
    uint32_t done_id[2][27];  // per stress component: evaluation already reduced
    uint32_t eval_seq;        // evaluations so far
    uint32_t nrec;            // series records so far
    uint32_t rec_base;        // nrec at the last reset of the means
    uint32_t health;          // H_* bits, sticky until read by the host
    uint32_t maxov_last_bits; // float bits: largest overlap of the last reduced evaluation
    uint32_t pad;
    double stress_sum[27];    // running sums for means
};

struct SysDyn {
    uint32_t halted;          // 1: some list may have expired; the remaining launches of the chunk do nothing
    uint32_t expire[2];       // 1: the integrate of the step with that parity found a particle whose
                              // displacement bound fails the list-validity test
    uint32_t list_need;       // largest neighbour count of a particle whose list overflowed at the
                              // last build (0: none overflowed); the host regrows the lists
    uint64_t rebuilds;
};

// Device buffers of one handle.  Particle arrays have npad entries, in
// Hilbert cell order; replicas are contiguous and padded to kTile.
// Per particle, for the half-pair kernel and its gather (one 16-byte record, so
// that a partner's lookup touches one line): bit e of im = entry e (a higher-id
// partner) interacts in the last evaluation; qoff = the particle's first pair within
// its wave's run (queue order); lo0 = first entry whose partner has the higher id
// (lists are sorted by id).
struct alignas(16) PairIdx {
    uint64_t im;
    uint32_t qoff;
    uint32_t lo0;
};

struct Bufs {
    uint32_t npad, nrep, nkeys_total, cap;   // cap = neighbour slots per particle
    int mixed;

    double4* pos;     // x, y, z, a
    double4* vh;      // half-step velocity (after kick 1) -- read by the pair kernel
    double4* wh;      // half-step angular velocity
    double4* vf;      // full-step velocity (after kick 2)
    double4* wf;
    void* F;          // double4 (FP64) or float4 (mixed)
    void* T;
    float4* vsh;      // mixed: FP32 copies of vh and wh used by pair gathers
    float4* wsh;
    uint32_t* id;

    // neighbour list, slot-major: nbr[e * npad + i]
    uint32_t* nbr;
    uint32_t* ncnt;
    // contact history per list entry, slot-major, canonical orientation (lower id first)
    void* hs;         // spring per entry: 3 doubles (3 floats in mixed precision), packed
    uint64_t* cmask;  // bit e: entry e holds a live contact
    uint64_t* smask;  // bit e: that contact slid at its last update
    // half-pair evaluation: each interacting pair is evaluated once, by its
    // lower-id particle, into its list entry; the higher-id particle reads it
    // through the mirror index
    PairIdx* pidx;    // per particle: interaction mask, queue offset, first higher-id entry
    uint8_t* mir;     // [e * npad + i], entry with a lower-id partner j: the entry of i in j's list
    void* pf;         // 3 doubles / 4 floats per pair: force on the lower-id particle; the pairs of
                      // the wave owning particles [64 w, 64 w + 64) sit in queue order
                      // (particles in order, entries in order) from 64 w * cap
    void* pt;         // same layout: torque on the lower-id particle (contact, or every pair
                      // with the rotational couplings)
    void* pt2;        // same layout: torque on the higher-id particle
    int rot;          // rotational lubrication couplings and pairwise Brownian torques on
    int ext;          // some model extension on (repulsion or the rotational couplings)

    // rebuild scratch
    uint32_t* key;        // cell key per particle
    uint32_t* cell_cnt;   // nkeys_total
    uint32_t* cell_fill;
    uint32_t* cell_start; // nkeys_total + 1
    uint32_t* scan_blk;   // block sums of the scan
    uint32_t* src;        // new slot -> old slot
    // carry of contact history across a rebuild: compact table per particle
    uint32_t* ct_id;      // [c * npad + i] partner id
    double* ct_s;         // [(c * 3 + d) * npad + i]
    uint8_t* ct_sl;       // sliding flag
    uint32_t* ct_n;
    // staging copies for the reorder
    double4* alt4[8];
    uint32_t* alt_id;

    // stress: per pair-kernel block partial sums (two parities), ring of per-step values
    double* partial;      // [parity][27][blk]
    float* ovpart;        // [parity][blk]: largest overlap seen by each pair-kernel block
    uint32_t nblk_max;    // pair-kernel blocks at 4 lanes per particle (partials per parity)
    double* ring;         // [rep][kRing][27]
    double* last;         // [rep][27]
    int lanes;            // pair kernel: lanes per particle (1, 2, 4)
    int ppb;              // particles per pair-kernel block (for the stress partials)
    int occ;              // half-pair kernel in FP64 without extensions: 1 = its form for occupancy
    uint32_t qcap;        // queue items per round of that form (2048; 64 under SIM_SMALL_QUEUE)

    // streaming autocorrelation of one recorded stress entry (Green-Kubo, Sec. IV.B):
    // acf_comp = entry 0..26 or -1 (off); per replica the last acf_nlag samples
    // (acf_hist, circular), the lag sums acf_sum[k] = sum_t s(t) s(t - k) and the
    // sample count acf_n
    int acf_comp;
    uint32_t acf_nlag;
    double* acf_hist;     // [rep][acf_nlag]
    double* acf_sum;      // [rep][acf_nlag]
    unsigned long long* acf_n;  // [rep]

    float* dacc;          // per particle: bound on its non-affine displacement since the last build
                          // (FP32, rounded up)
    double4* disp;        // per particle: accumulated non-affine displacement (x, y, z) since the
                          // creation, the last state upload or sim_reset_displacement
    float* dpart;         // [parity][kTile-block]: largest dacc of the block after that step's drift
    uint32_t* blk_rep;    // replica of each kTile-block of particles
    RepParams* reps;
    RepDyn* dyn;
    SysDyn* sys;
};

constexpr int kRing = 8192;
constexpr int kCtCap = 16;   // contacts per particle carried across a rebuild

// kernel launchers (susp_kernels.hip).  q is the parity of the step being taken
// (or, for an evaluation without a step, of the current step).
// kick 1 + drift + wrap of a step; also reduces the stress of the previous step
void launch_integrate(const Bufs& b, hipStream_t st, int q);
// forces of a step (advance = 1: next step counter and offset, list-expiry test,
// kick 2 if kick) or of the current state (advance = 0); only_rep: one replica
// or 0xFFFFFFFF
// kev: null, or events {pair start, pair end, gather start, gather end} that the
// hardware records when those kernels start and end (the gather pair only with the
// half-pair variant); fuse (half-pair variant only): the gather also takes kick 1
// and the drift of the next step, which then needs no integrate launch
void launch_pair_force(const Bufs& b, hipStream_t st, int q, int kick, int advance, uint32_t only_rep,
                       const hipEvent_t* kev = nullptr, int fuse = 0);
// reduces pending stress partials of parity q
void launch_finalize(const Bufs& b, hipStream_t st, int q);
// The neighbour lists and mirror index again from the cells and the carried
// contact history of the last rebuild (after the lists were regrown); q, in_step as
// for launch_rebuild.
void launch_relist(const Bufs& b, hipStream_t st, int q, int in_step);
// Rebuild of cells and neighbour lists from the current positions; q is the
// parity of the next force evaluation.  in_step: called between kick 1 and the
// force evaluation of a step.  ct_input_rep: 0xFFFFFFFF = carry contact
// history from the current lists; 0xFFFFFFFE = every replica takes the
// host-written compact table; else that replica does.
void launch_rebuild(const Bufs& b, hipStream_t st, int q, int in_step, uint32_t ct_input_rep);
// kinetic sums of one replica (m |v - U^inf|^2 and I |w - Omega^inf|^2): nblk = n_pad / 256 blocks, 2 doubles each
void launch_kinetic(const Bufs& b, hipStream_t st, uint32_t rep, uint32_t nblk, double* part);
// mean-square displacement sums of one replica: nblk = n_pad / 256 blocks, 3 doubles each
void launch_msd(const Bufs& b, hipStream_t st, uint32_t rep, uint32_t nblk, double* part);
// pair histograms of one replica at parity p from a cell pass reaching `reach`:
// mode 0 = distances r < r_max in nbins bins; mode 1 = the flow-gradient slice
// |r_z| < slab / 2 on an nbins x nbins grid over [-r_max, r_max)^2 (each pair at r and -r)
void launch_rdf(const Bufs& b, hipStream_t st, int p, uint32_t rep, uint32_t nblk, int mode, double r_max,
                double slab, double reach, uint32_t nbins, unsigned long long* counts);
// zeroes n 64-bit words with a kernel
void launch_zero64(hipStream_t st, unsigned long long* a, uint32_t n);
// The scratch array of the entry points that allocate nothing: kScratchWords 64-bit words,
// a static device array, one copy per GPU.  Returns the current device's copy (its address
// looked up on first use on that device), or null with a message in err.
constexpr uint32_t kScratchWords = 1u << 16;
constexpr int kMaxDevices = 64;
unsigned long long* scratch_ptr(std::string& err);
// autocorrelation of one recorded stress component of one replica over the records
// [first, first + count) of the ring: out[lag] = mean_t s(t) s(t + lag), lag < nlag
void launch_acf(const Bufs& b, hipStream_t st, uint32_t rep, int comp, uint32_t first, uint32_t count,
                uint32_t nlag, double* out);
// structural Brownian stress sums of one replica at parity p: nblk = n_pad / 256
// blocks, 9 doubles each into part
void launch_struct(const Bufs& b, hipStream_t st, int p, uint32_t rep, uint32_t nblk, double* part);
void launch_diag(const Bufs& b, hipStream_t st, int p, uint32_t rep, uint32_t n, uint32_t* out_ij, double* out_s,
                 int32_t* out_sl, uint32_t* count, uint32_t cap, int mode);

}  // namespace susp
