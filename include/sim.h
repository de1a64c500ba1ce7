/*
 * sim.h -- C ABI of the MI355X (gfx950) force engine for sheared dense
 * suspensions: the per-timestep hot path of the pairwise model of Li, Royer &
 * Ness (arXiv 2307.13802).
 *
 * One handle holds R >= 1 independent replicas (systems) that advance
 * together; every stage of a step is one kernel launch over all replicas.
 * Per replica and per step the library computes, on the GPU:
 *   - the Lees-Edwards offset and the wrap of particles into the sheared
 *     periodic box (Sec. II.E: the tilted box remapped at strain +-1/2 is the
 *     same image lattice as a Lees-Edwards offset);
 *   - a Verlet neighbour list from Hilbert-ordered cells, rebuilt on device when
 *     the accumulated non-affine displacement can have used up the skin
 *     (Sec. II, footnote on the skin);
 *   - per pair: the squeeze and shear lubrication force of eq. (force_lub)
 *     with X^A_11, Y^A_11 (Sec. II.B), regularised at xi_min and cut off above
 *     xi_cut; the Hookean normal and frictional tangential contact force and
 *     torque of eq. (force_contact), (torque_contact) with per-pair spring
 *     history and Coulomb limit mu (Sec. II.A); the pairwise Brownian force of
 *     eq. (force_brownian_lub) with amplitude sqrt(2 kT/dt) (Sec. II.C);
 *   - per particle: Stokes drag force and torque, eq. (force_drag),
 *     (torque_drag), and one-body Brownian force and torque, eq.
 *     (force_brownian_drag), (torque_brownian_drag);
 *   - velocity-Verlet for translation and rotation (Sec. II, I = 2/5 m a^2);
 *   - the virial stresses -F (x) r / V of contact, lubrication and Brownian
 *     pair forces (Sec. II.A, II.B, II.D), accumulated in FP64, the drag
 *     stresslet (Sec. II.B) and the total stress (Sec. IV.D).
 *
 * Conventions
 *   Units are the paper's (Sec. II.E): lengths in a, masses in rho a^3, time
 *   such that k_n = 1 gives unit frequency.  Particle ids are 0..n-1 in the
 *   order of the arrays given to sim_create.  x is the flow direction, y the
 *   gradient direction, z the vorticity direction; U^inf = gammadot (y - Ly/2)
 *   e_x and Omega^inf = (0, 0, -gammadot/2).  r_ij = x_i - x_j (minimum
 *   image), so n_ij points from j to i.  Arrays of vectors are particle-major,
 *   xyz interleaved (x0 y0 z0 x1 ...).  Stress tensors are 3x3 row-major,
 *   element [a][b] = -(1/V) sum F_a r_b.
 *
 * Memory and threading
 *   The caller owns every host array; inputs are copied, outputs are written
 *   into caller-sized buffers.  The library owns the handle and all device
 *   memory (through the allocator set by sim_set_allocator, else hipMalloc).
 *   All GPU work is ordered on the stream given at creation.  A handle is not
 *   thread safe; different handles are independent.
 *
 * Determinism
 *   No floating-point atomics are used.  Trajectories (positions, velocities,
 *   forces, torques, springs, interaction sets) are bit-identical for the same
 *   build, inputs and configuration whatever launch parameters the tuner picks
 *   (lanes per particle, kernel form, skin, cell size): each particle's terms
 *   are summed in a fixed item order.  The stress sums run over the pairs in an
 *   order that follows the launch shape, so with tuned parameters their last
 *   bits can differ between two creations; they are bit-identical when the
 *   parameters are the same (fixed in the configuration, or read from the
 *   cache set by sim_set_tune_cache; sim_stats reports the set in use).
 *
 * Errors
 *   Every function returns an int32 status: 0 = SIM_OK, negative = error.
 *   sim_strerror gives a static description of a code and sim_last_error the
 *   message of the last failure on a handle.  No exception crosses the ABI.
 */
#ifndef SUSP_SIM_H
#define SUSP_SIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SIM_OK         0
#define SIM_EINVAL    -1  /* bad configuration or argument                         */
#define SIM_ENOMEM    -2  /* device or host allocation failed                       */
#define SIM_EDEVICE   -3  /* HIP runtime error (text in sim_last_error)              */
#define SIM_EUNSTABLE -4  /* NaN/Inf force or overlap above the limit (see below)    */
#define SIM_ECAPACITY -5  /* neighbour list capacity exceeded                        */
#define SIM_ERANGE    -6  /* replica index out of range or output buffer too small   */

/* precision of the pair arithmetic */
#define SIM_FP64  0       /* everything in FP64                                      */
#define SIM_MIXED 1       /* FP64 positions, image offsets, gaps, stress and
                             integration; FP32 pair forces with compensated sums     */

/* sim_config.flags (test and measurement switches; 0 = the physical model) */
#define SIM_FREEZE_X          0x001u /* positions are not advanced                   */
#define SIM_NO_LUB            0x002u /* drop the lubrication force                   */
#define SIM_NO_PAIR_BROWN     0x004u /* drop the pairwise Brownian force             */
#define SIM_NO_CONTACT        0x008u /* drop contact force and torque                */
#define SIM_NO_ONEBODY        0x010u /* drop one-body drag and Brownian terms        */
#define SIM_LUB_ROT           0x020u /* model switch: add the rotational lubrication
                                        couplings Y^B, Y^C to the pair force and torques
                                        (eq. force_lub, torque_lub1, torque_lub2) and the
                                        pairwise Brownian torques (eq. torque_brownian_lub1,
                                        torque_brownian_lub2); half-pair kernel only       */
#define SIM_REBUILD_EACH_STEP 0x100u /* rebuild the neighbour list every step        */
#define SIM_NO_GRAPH          0x200u /* launch kernels directly, no HIP graph        */
#define SIM_HALF_OCC_ON       0x400u /* FP64, no model switch: use the pair kernel's form
                                        for occupancy (the pair queue in rounds, part of
                                        the stress sums in LDS, 3 waves per SIMD) rather
                                        than choosing by timing at creation; the same
                                        trajectories bit for bit                        */
#define SIM_HALF_OCC_OFF      0x800u /* ... never use that form                       */
#define SIM_TRACK_DISPLACEMENT 0x2000u /* accumulate each particle's non-affine
                                        displacement (sim_displacement, sim_msd): 64
                                        bytes of HBM traffic per particle and step, so
                                        off unless asked for; no trajectory changes     */
#define SIM_SMALL_QUEUE      0x1000u /* test switch: that form processes its pair queue
                                        64 items per round (instead of 2048), so that
                                        every wave takes several rounds                 */

/* sim_stress components and modes */
#define SIM_STRESS_CONTACT 0      /* -(F^C + F^R) (x) r / V: contact and
                                     short-ranged repulsion       (Sec. II.A, IV.F) */
#define SIM_STRESS_LUB     1      /* -F^{H,L} (x) r / V                 (Sec. II.B) */
#define SIM_STRESS_BROWN   2      /* -F^{B,L} (x) r / V, instantaneous  (Sec. II.D) */
#define SIM_STRESS_DRAG    3      /* (1/V) sum 20/3 pi eta a^3 E        (Sec. II.B);
                                     0 under SIM_NO_ONEBODY (no drag)                */
#define SIM_STRESS_TOTAL   4      /* contact + lubrication + drag       (Sec. IV.D);
                                     its xy entry / (eta gammadot) is eta_r (II.E)  */
#define SIM_STRESS_LAST    0      /* value at the last evaluated step               */
#define SIM_STRESS_MEAN    1      /* mean over steps since sim_reset_stress/create  */

typedef struct sim sim;

/* One replica.  struct_size must equal sizeof(sim_config). */
typedef struct sim_config {
    uint32_t struct_size;
    uint32_t n;             /* particles, 1 <= n < 2^32 - 1                          */
    double   box[3];        /* Lx, Ly, Lz                                            */
    double   rho;           /* particle density (mass / length^3), Sec. II.E        */
    double   eta;           /* fluid viscosity, Sec. II.B                            */
    double   kn, kt;        /* normal and tangential contact stiffness, Sec. II.A   */
    double   mu;            /* static friction coefficient, Sec. II.A                */
    double   kT;            /* thermal energy, Sec. II.C                             */
    double   gammadot;      /* shear rate (x velocity varying along y)               */
    double   dt;            /* time step                                             */
    double   xi_cut;        /* no lubrication for dimensionless gaps xi > xi_cut     */
    double   xi_min;        /* xi is replaced by xi_min when smaller (Sec. II.B)     */
    double   skin;          /* Verlet skin, length; 0 selects 0.2 * min radius; < 0:
                               the tuner picks 0.1 ... 0.4 * min radius              */
    double   le_offset0;    /* initial Lees-Edwards offset (x shift of the y image)  */
    double   max_overlap;   /* health limit on the overlap; <= 0 selects 0.1 * min a */
    double   repulsion;     /* A >= 0 of the short-ranged repulsion (A / kappa)
                               exp(-h / kappa) n, kappa = 0.01 (a_i + a_j) (Sec.
                               IV.F), on the pairs with gap h <= 16 kappa (where it
                               has decayed to e^-16; the paper states no cut-off);
                               0 = none                                              */
    double   cell_factor;   /* search cells at least cell_factor times the list range
                               wide: 0 selects 1, < 0 the tuner picks 1, 1.5 or 2;
                               else in [1, 4]                                        */
    uint64_t seed;          /* key of the counter-based noise generator             */
    uint64_t step0;         /* step counter of the initial state                     */
    int32_t  precision;     /* SIM_FP64 or SIM_MIXED, identical for all replicas     */
    uint32_t flags;         /* SIM_* flags, identical for all replicas               */
    uint32_t nlist_cap;     /* initial neighbour list capacity per particle (0
                               selects 48); a build that finds more partners within
                               the list range regrows the lists to hold them, up to
                               64 (beyond: SIM_ECAPACITY)                            */
    uint32_t lanes;         /* lanes sharing one particle's list in the pair kernel
                               (1, 2 or 4: 64, 32 or 16 particles per wave); 0 =
                               chosen by timing at creation                          */
    uint32_t pair_kernel;   /* SIM_KERNEL_AUTO or SIM_KERNEL_HALF (the same kernel)   */
    uint32_t reserved;      /* must be 0                                             */
} sim_config;

/* sim_config.pair_kernel: every interacting pair is evaluated once, by its
 * lower-id particle (`lanes` lanes per particle test its list), packed 64 to a
 * wave; a second launch sums each particle's pair terms and one-body terms in
 * item order */
#define SIM_KERNEL_AUTO  0
#define SIM_KERNEL_HALF  3

typedef struct sim_stats_t {
    double  contacts_per_particle;  /* Z = 2 * contacts / n                          */
    double  sliding_fraction;       /* contacts at the Coulomb limit / contacts       */
    double  max_overlap;            /* largest overlap at the last evaluation          */
    double  neighbours_per_particle;/* Verlet list entries per particle              */
    double  interacting_per_particle; /* pairs with xi <= xi_cut, counted per side     */
    int64_t contacts;               /* number of contacts (pairs with overlap)         */
    int64_t rebuilds;               /* neighbour list builds since creation            */
    int64_t steps;                  /* steps taken since creation                      */
    uint64_t step;                  /* current step counter                            */
    double  le_offset;              /* current Lees-Edwards offset                     */
    int32_t lanes;                  /* lanes per particle used by the pair kernel       */
    int32_t pair_kernel;            /* SIM_KERNEL_HALF                                   */
    int32_t occupancy_form;         /* 1: the pair kernel's form for occupancy is in use
                                       (see SIM_HALF_OCC_ON), 0 otherwise               */
    int32_t tune_source;            /* launch and list parameters: 0 configured or
                                       default, 1 measured at creation, 2 read from the
                                       cache (sim_set_tune_cache)                        */
    double  skin;                   /* Verlet skin of the replica (length)               */
    double  cell_factor;            /* search cells >= cell_factor x the list range      */
    double  kT_translational;       /* sum m |v - U^inf(x)|^2 / (3 n): the temperature of
                                       the peculiar translational motion (full-step v)   */
    double  kT_rotational;          /* sum I |w - Omega^inf|^2 / (3 n), rotational       */
    int32_t cells_x, cells_y, cells_z; /* search cells per box side                     */
    int32_t list_cap;               /* entries per particle the lists hold now: nlist_cap,
                                       grown when a build finds more partners (to 64)   */
} sim_stats_t;

/* Checks a configuration and its radii on the host (no GPU needed).
 * radii: n doubles, host memory.  Returns SIM_EINVAL for both SIM_HALF_OCC_ON
 * and SIM_HALF_OCC_OFF, SIM_HALF_OCC_ON with SIM_MIXED, SIM_LUB_ROT or
 * repulsion > 0, a pair_kernel other than 0 and SIM_KERNEL_HALF, n = 0, a <= 0,
 * dt <= 0, rho/eta <= 0, kn/kt < 0, mu < 0, kT < 0, repulsion < 0, xi_min <= 0,
 * xi_min >= xi_cut, a box side not larger than twice the largest
 * interaction range plus skin (the minimum image must be unique; with a tuned
 * skin, the smallest candidate), a wrong struct_size, nlist_cap > 64, lanes
 * not in {0, 1, 2, 4}, cell_factor in (0, 1) or above 4, or a nonzero
 * reserved field. */
int sim_validate(const sim_config* cfg, const double* radii);

/* Tuned launch and list parameters are read from and added to the cache file at
 * path (a JSON object keyed by device, precision, model switches, the fixed
 * parameters and buckets of particle count, volume fraction, size ratio and
 * Peclet number) by the creations that follow; NULL or "" = no cache (the
 * default).  A cached set is used without measuring, so that a rerun has the same
 * parameters; a cache that cannot be read or written is ignored. */
int sim_set_tune_cache(const char* path);

/* Creates a handle with n_replicas systems.  For replica r: radii[r] -> n
 * doubles; x0[r] -> 3n doubles inside [0, L); v0[r], w0[r] -> 3n finite doubles
 * of velocities and angular velocities, or NULL for U^inf(x) and Omega^inf
 * (a coordinate outside [0, L) or a NaN or infinity: SIM_EINVAL).
 * hip_stream is a hipStream_t (NULL = the null stream).  Evaluates the forces
 * of every replica at its initial state (Sec. II force law at step step0,
 * using v0 and w0), so the first sim_step starts a velocity-Verlet step.
 * On success *out receives the handle. */
int sim_create(const sim_config* cfgs, int32_t n_replicas, const double* const* radii,
               const double* const* x0, const double* const* v0, const double* const* w0,
               void* hip_stream, sim** out);

/* Advances every replica by nsteps velocity-Verlet steps (Sec. II): half
 * kick, drift, Lees-Edwards wrap, neighbour rebuild when needed, forces at
 * the new positions with the half-step velocities, half kick.  Returns after
 * the work is complete.  SIM_EUNSTABLE / SIM_ECAPACITY report a step whose
 * forces are not trustworthy; the state is then that of the failing step. */
int sim_step(sim* s, int64_t nsteps);

/* Stress of one replica (3x3 row-major, FP64, host memory). */
int sim_stress(sim* s, int32_t replica, int32_t component, int32_t mode, double out[9]);

/* Restarts the running means used by SIM_STRESS_MEAN for all replicas. */
int sim_reset_stress(sim* s);

/* Per-step series of the contact, lubrication and Brownian stresses (27
 * doubles per step: [component][a][b]) recorded since the previous call, at
 * most the ring capacity (8192 steps); oldest first.  *count receives the
 * number of steps available; if it exceeds cap, SIM_ERANGE is returned and
 * nothing is consumed. */
int sim_stress_series(sim* s, int32_t replica, double* out, int64_t cap, int64_t* count);

/* Structural Brownian stress of the current configuration of one replica
 * (Sec. II.D): -(kT / V) sum_i (a_i / Delta_i) sum_{j in shell of i}
 * n_ij (x) n_ij, with the shell of i the partners whose gap
 * h = |r| - (a_i + a_j) is at most Delta_i = 0.05 a_i (contacts included).
 * It is not part of the total stress.  Rebuilds the neighbour lists first
 * (which changes no trajectory).  3x3 row-major, FP64, host memory.
 * SIM_EINVAL if the list range cannot cover the shell (skin + (a_i + a_j)
 * xi_cut / 2 < 0.05 a_max for some pair). */
int sim_structural_stress(sim* s, int32_t replica, double out[9]);

/* Analysis of the trajectories (Sec. III), computed on the device.
 *
 * sim_displacement: each particle's accumulated non-affine displacement
 * (the drift of every step minus the imposed flow integrated along it; the
 * plain unwrapped displacement when gammadot = 0) since sim_create,
 * sim_set_state of its replica or sim_reset_displacement; id order, 3n
 * doubles.  sim_msd: its mean square per axis, out[3] = <dx^2>, <dy^2>,
 * <dz^2> over the replica's particles (the MSD of Sec. III.B).
 * sim_reset_displacement: zero for every replica.  All three need a handle
 * created with SIM_TRACK_DISPLACEMENT (else SIM_EINVAL). */
int sim_displacement(sim* s, int32_t replica, double* out_3n);
int sim_msd(sim* s, int32_t replica, double out[3]);
int sim_reset_displacement(sim* s);

/* Histogram of the pair distances r = |r_ij| < r_max of the current
 * configuration of one replica (each pair once; minimum image in the sheared
 * box), nbins bins of width r_max / nbins, from a cell pass of its own (not the
 * neighbour lists): counts receives nbins integers.  Dividing by the ideal-gas
 * count of each shell gives g(r) (Sec. III.A), e.g. out to the flat region of
 * the potential of mean force.  Rebuilds the neighbour lists first (which
 * changes no trajectory).  SIM_EINVAL for nbins outside [1, 2^24] or r_max
 * outside (0, L/2), L the smallest box side. */
int sim_rdf(sim* s, int32_t replica, double r_max, int32_t nbins, uint64_t* counts);

/* sim_rdf for callers that cannot allocate device memory (code under HIP graph
 * capture, tight sampling loops, harnesses that forbid hipMalloc): the same
 * histogram, bit for bit, with its bins in a static device array of the library
 * (65,536 64-bit words per GPU, held until the process ends) instead of memory
 * allocated per call; it calls no hipMalloc, hipFree or other allocating routine
 * (a list build of the call that finds more partners than the lists hold leaves
 * their regrow to the next call that uses them).  The bins are cleared by a
 * kernel at every call.  All calls on one GPU share
 * that array: calls that overlap in time on one GPU (from several threads or
 * streams) race and must be serialised by the caller.  SIM_EINVAL for nbins
 * outside [1, 65536] and as sim_rdf otherwise; SIM_EDEVICE if the array's
 * address cannot be obtained on the current device. */
int sim_rdf_noalloc(sim* s, int32_t replica, double r_max, int32_t nbins, uint64_t* counts);

/* Slice of the pair distribution through the flow-gradient (xy) plane of one
 * replica (Sec. IV.D, the microstructure under shear): pairs with
 * |r_z| < slab / 2 and |r_x|, |r_y| < r_max, counted at r_ij and at -r_ij on an
 * nbins x nbins grid over [-r_max, r_max)^2; counts[ix * nbins + iy], ix along
 * x (flow), iy along y (gradient).  Dividing by the ideal-gas count of a bin
 * (n (n - 1) / V x bin area x slab) gives g in the slice.  Rebuilds the lists
 * first.  SIM_EINVAL for nbins outside [1, 4096], slab <= 0 or
 * sqrt(2 r_max^2 + slab^2 / 4) not in (0, L/2). */
int sim_rdf_xy(sim* s, int32_t replica, double r_max, double slab, int32_t nbins, uint64_t* counts);

/* Time autocorrelation of one recorded stress component (component
 * SIM_STRESS_CONTACT, _LUB or _BROWN, entry alpha, beta in 0..2) for Green-Kubo
 * integrals (Sec. IV.B): out[k] = mean over t of S(t) S(t + k), k < nlag, over
 * the count - k pairs of records.  If sim_stress_acf_stream is accumulating
 * this entry with at least nlag lags, the sums cover every record since the
 * stream started or sim_reset_stress (no limit on the count); otherwise the
 * records since sim_reset_stress in the ring (at most the last 8192).
 * SIM_ERANGE if fewer than nlag records are available. */
int sim_stress_acf(sim* s, int32_t replica, int32_t component, int32_t alpha, int32_t beta, int64_t nlag,
                   double* out);

/* Starts accumulating the autocorrelation of one stress entry (as in
 * sim_stress_acf) for every replica on the device, at every recorded step, for
 * lags 0..nlag-1 (nlag <= 2^20): no record ring bounds the run length.  The
 * sums restart with sim_reset_stress; nlag = 0 stops the stream.  Each lag's sum
 * runs in time order. */
int sim_stress_acf_stream(sim* s, int32_t component, int32_t alpha, int32_t beta, int64_t nlag);

/* Positions of one replica in id order, wrapped into [0, L), FP64, 3n doubles. */
int sim_positions(sim* s, int32_t replica, double* out_3n);

/* Full state of one replica in id order (any pointer may be NULL):
 * positions, full-step velocities and angular velocities, last force and
 * torque, Lees-Edwards offset and step counter. */
int sim_get_state(sim* s, int32_t replica, double* x, double* v, double* w, double* F, double* T,
                  double* le_offset, uint64_t* step);

/* Replaces the state of one replica.  x, v, w: 3n doubles (required; x inside
 * [0, L), every value given here finite, else SIM_EINVAL).
 * c_ij: n_contacts (id_i, id_j) pairs with id_i < id_j and c_s their springs
 * (3 doubles each); pairs that are not overlapping are ignored.  If F and T
 * are given they are taken as the forces of the state (a restart); if both
 * are NULL the forces are evaluated at this state with these velocities at
 * step counter `step` (forces of the other replicas are left unchanged). */
int sim_set_state(sim* s, int32_t replica, const double* x, const double* v, const double* w,
                  const double* F, const double* T, double le_offset, uint64_t step,
                  const uint32_t* c_ij, const double* c_s, int64_t n_contacts);

/* Last evaluated force and torque of one replica, id order, 3n doubles each. */
int sim_forces(sim* s, int32_t replica, double* F_3n, double* T_3n);

/* Interaction set of the last evaluation: pairs (id_i < id_j) with
 * dimensionless gap xi <= xi_cut, sorted.  cap is in pairs. */
int sim_pairs(sim* s, int32_t replica, uint32_t* ij_2m, int64_t cap, int64_t* count);

/* Verlet set of the current neighbour list (|r| <= (a_i + a_j)(1 + xi_cut/2)
 * + skin at the last rebuild; with the repulsion on, (a_i + a_j)(1 + 16 x 0.01)
 * + skin when that is larger), pairs (id_i < id_j), sorted. */
int sim_nlist(sim* s, int32_t replica, uint32_t* ij_2m, int64_t cap, int64_t* count);

/* Contact history: pairs (id_i < id_j) in contact at the last evaluation,
 * their springs s_ij (3 doubles) and whether they slid (Coulomb limit). */
int sim_contacts(sim* s, int32_t replica, uint32_t* ij_2m, double* s_3m, int32_t* sliding,
                 int64_t cap, int64_t* count);

/* Statistics of one replica at the last evaluation (the kinetic temperatures
 * measure the equipartition of Sec. II.C: each tends to kT at rest). */
int sim_stats(sim* s, int32_t replica, sim_stats_t* out);

/* Kernel timing: when enabled, sim_step launches directly (no graph), in the
 * same sequence as the graphs, in batches of up to 32 steps without a host
 * wait, and each force kernel with HIP events that the hardware records when
 * the kernel starts and ends (on the library stream).  sim_kernel_time returns
 * the number of timed steps and the total duration, in milliseconds since the
 * last enable, of their force evaluations (all pair-force launches); a batch
 * in which a list expiry halted a step is not counted.  sim_stage_time gives
 * one stage: 0 = the integrate launches (with SIM_KERNEL_HALF one per batch:
 * the gathers integrate the other steps), 1 = the pair kernel, 2 = the gather
 * of SIM_KERNEL_HALF (0 for the other variants, whose pair kernel includes
 * it); SIM_EINVAL for another stage. */
int sim_profile(sim* s, int32_t enable);
int sim_kernel_time(sim* s, int64_t* launches, double* total_ms);
int sim_stage_time(sim* s, int32_t stage, int64_t* launches, double* total_ms);

/* Destroys a handle and frees its device memory. */
int sim_destroy(sim* s);

/* Static description of a status code. */
const char* sim_strerror(int32_t code);

/* Copies the message of the last error on the handle (or the last
 * handle-less error if s is NULL) into buf (NUL-terminated). */
int sim_last_error(const sim* s, char* buf, size_t len);

/* Routes device allocations of handles created afterwards through alloc/free
 * (e.g. a framework's caching allocator); NULL restores hipMalloc/hipFree. */
int sim_set_allocator(void* (*alloc_fn)(size_t bytes, void* ctx), void (*free_fn)(void* p, void* ctx),
                      void* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SUSP_SIM_H */
