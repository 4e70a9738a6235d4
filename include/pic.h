/*
 * pic.h -- C ABI of libpic, the MI355X (gfx950) hot path of a 1D3V
 * electrostatic Particle-in-Cell Monte Carlo (PIC-MC) time step.
 *
 * The operations follow the explicit PIC cycle of Williams et al., arXiv
 * 2404.10270, Sec. 2 (five phases: plasma density calculation, density
 * smoother, field solver, collisions and plasma-wall interaction, particle
 * mover), the mover statements of its moveb listing (Sec. 6), and its Table 1
 * test case (Sec. 3.4: electrons, ions and kinetic neutral atoms, no field
 * solver, ionisation depleting the gas).
 *
 * Units.  Particle positions are in cells (domain [0, nc)), velocities in
 * cells per step; the configuration carries SI (or plasma-unit) physical
 * inputs and libpic converts them once in pic_init.
 *
 * Ownership.  Every device buffer is allocated by the caller (typically as
 * PyTorch tensors) with the sizes pic_query_sizes reports, stays owned by the
 * caller, and must outlive the context.  libpic never allocates or frees
 * device memory; a context holds host metadata only.  The one exception is
 * the static workspace array of pic_init_static (a fixed-size device array
 * of the library, not an allocation at run time).
 *
 * Streams.  pic_init synchronises its stream once, after uploading the
 * tables (the initial draw, sort, deposit and field solve it enqueues after
 * that are not waited for); pic_diagnostics, pic_autotune_sort and
 * pic_autotune synchronise too.  Every other phase call enqueues
 * work on the HIP stream given to pic_init and returns without
 * synchronising; pic_query_sizes, pic_region, pic_destroy and pic_strerror
 * do no device work.  A context is not thread-safe; use one context per
 * stream.
 *
 * Errors.  Host-detectable errors (bad arguments or configuration) return a
 * negative pic_status before any device work is enqueued.  Conditions found
 * on the device (capacity overflow, |vx| >= 1 cell/step, non-finite values)
 * set bits of a device status word, reported by the next pic_diagnostics.
 * No exception or abort crosses the ABI.
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_MAX_SPECIES 4
#define PIC_FRAC_BITS 32          /* fixed-point fraction bits of the deposit */

typedef enum {
    PIC_OK = 0,
    PIC_E_ARG = -1,        /* null pointer, bad count, misaligned buffer */
    PIC_E_CONFIG = -2,     /* invalid physical or numerical configuration */
    PIC_E_DEVICE = -3,     /* a HIP call failed */
    PIC_E_CAPACITY = -4,   /* device status: a created/uploaded particle did not fit */
    PIC_E_CFL = -5,        /* device status: |vx| >= 1 cell per step */
    PIC_E_NONFINITE = -6,  /* device status: non-finite velocity or field */
    PIC_E_STATE = -7,      /* call out of order (e.g. a phase before pic_init) */
    PIC_E_SCRATCH = -8,    /* pic_init_static: the workspace exceeds PIC_STATIC_WORK_MAX */
    PIC_E_BUSY = -9        /* pic_init_static: a live context holds the device's static workspace */
} pic_status;

/* device status word bits (pic_diag.status) */
#define PIC_ST_CAPACITY   0x1u
#define PIC_ST_CFL        0x2u
#define PIC_ST_NONFINITE  0x4u
#define PIC_ST_CANDIDATES 0x8u   /* the collision candidate or event list overflowed */
#define PIC_ST_INTERNAL   0x10u  /* a device-side consistency check failed */
#define PIC_ST_BAD_INIT   0x20u  /* an uploaded particle was out of range and was dropped */
#define PIC_ST_NN_CAP     0x40u  /* a local kinetic-neutral density exceeded the bound n_n */

typedef enum { PIC_BC_PERIODIC = 0, PIC_BC_ABSORB = 1 } pic_bc;
/* PIC_KIND_NEUTRAL: kinetic neutral atoms (q = 0), moved ballistically and
 * consumed by electron-impact ionisation (at most one such species) */
typedef enum { PIC_KIND_ELECTRON = 0, PIC_KIND_ION = 1, PIC_KIND_NEUTRAL = 2 } pic_kind;
typedef enum {
    PIC_FP32 = 0,   /* FP32 gather/push, (cell, f32 in-cell offset) positions, fixed-point deposit */
    PIC_FP64 = 1    /* FP64 gather/push, f64 positions in cells, fixed-point deposit */
} pic_precision;

typedef struct {
    double q;           /* charge [C] */
    double m;           /* mass [kg] */
    double w;           /* real particles per macro-particle per unit area [m^-2] */
    int32_t kind;       /* pic_kind: selects the collision processes */
    int32_t nstep;      /* subcycling (nstep of the moveb listing, Sec. 6): pushed on steps
                           s with s mod nstep = 0 over nstep dt, deposited every step;
                           0 or 1 = every step */
    int64_t capacity;   /* particle slots reserved for this species */
    int64_t n_init;     /* initial particles: uploaded into buffer set 0 before pic_init,
                           or drawn there by pic_init with PIC_INIT_DEVICE */
    double v_cap;       /* speed bounding the null-collision frequency [m/s] */
    double T_src;       /* temperature of source-born particles [J] */
    double T_init;      /* temperature of the drawn initial Maxwellian [J] (PIC_INIT_DEVICE) */
} pic_species;

typedef struct {
    int32_t nc;          /* cells; nodes 0..nc */
    int32_t bc;          /* pic_bc */
    int32_t nsp;         /* species, 1..PIC_MAX_SPECIES */
    int32_t precision;   /* pic_precision (must agree across instances) */
    int32_t mcc_on;      /* null-collision MCC (needs one electron and one ion species;
                            with a neutral species its atoms are the collision targets) */
    int32_t source_on;   /* pair source refilling the ions lost to the walls */
    int32_t _pad0, _pad1;
    uint64_t seed;       /* key of the Philox draws */
    double dx, dt, eps0; /* cell size [m], time step [s], permittivity [F/m] */
    double B0;           /* magnetic field magnitude [T] */
    double theta;        /* angle of B to the wall normal x, in the x-y plane [rad] */
    pic_species sp[PIC_MAX_SPECIES];
    double n_n, T_n;     /* neutral density [m^-3] (with a kinetic neutral species: the
                            bound of its local density in the null-collision test)
                            and temperature [J] */
    double sig_el, sig_iz, E_iz, sig_cx;  /* cross sections [m^2], threshold [J] */
    uint64_t next_id;    /* id given to the first created particle */
    int64_t step0;       /* index of the first step (keys the draws) */
    /* drawn initial state (PIC_INIT_DEVICE only) */
    double init_amp;     /* amplitude A of the electron density perturbation */
    int32_t init_mode;   /* its mode number m */
    uint32_t init_opts;  /* PIC_INIT_OPT_* */
    /* density smoother (Sec. 2, phase 2): passes of the binomial (1,2,1)/4
       filter on the node charges rho_j V_j before the field solve; at an
       absorbing wall the quarter that would leave stays on the wall node
       (total charge unchanged), a periodic grid wraps.  0 = off, at most 64. */
    int32_t smooth_passes;
    int32_t _pad2;
    /* electron-impact excitation: cross section [m^2] and threshold [J]
       (the electron loses E_ex and leaves isotropically) */
    double sig_ex, E_ex;
    /* no field solve (E = 0), as in the Table 1 case: the deposit, rho and
       the neutral density are still formed */
    int32_t field_off;
    uint32_t xs_flags;   /* PIC_XS_* */
} pic_config;

/* ionisation with a constant rate coefficient sig_iz * v_cap (frequency
   n sig_iz v_cap whatever the speed) instead of a constant cross section */
#define PIC_XS_IZ_RATE 0x1u

/* options of the drawn initial state */
#define PIC_INIT_OPT_QUIET 0x1u  /* lattice positions (p + 1/2) nc / n instead of uniform draws */
#define PIC_INIT_OPT_PAIR  0x2u  /* a species with species 0's count starts at its positions */

typedef struct {
    int64_t n_slots;     /* particle slots per array of one buffer set */
    int64_t n_segments;  /* n_inst * nsp */
    int64_t n_nodes;     /* grid nodes over all instances: sum(nc_i + 1) */
    uint64_t work_bytes; /* size of the device workspace */
    int64_t x_elem_bytes;/* 4 (PIC_FP32: float offset) or 8 (PIC_FP64: double position) */
    int64_t v_elem_bytes;/* 4 or 8 */
    int64_t mover_blocks;     /* default persistent grid of the movers (one residency on 256 CUs) */
    int64_t mover_blocks_max; /* the largest grid pic_set_mover accepts */
} pic_sizes;

/*
 * Particle buffers: two sets (b = 0, 1) of structure-of-arrays, each array
 * n_slots long, 256-byte aligned.  Segment s = inst * nsp + species occupies
 * slots [seg_base[s], seg_base[s+1]) of every array (seg_base from
 * pic_query_sizes).  Set 0 holds the initial state: the n_init particles of
 * a segment are its first n_init slots.  The current set changes when
 * pic_sort compacts into the other one; pic_diagnostics reports it.
 *   x   PIC_FP32: float in-cell offset f in [0,1); PIC_FP64: double x in cells
 *   cell int32 cell index (PIC_FP32 only; NULL for PIC_FP64)
 *   vx, vy, vz float (PIC_FP32) or double (PIC_FP64), cells per step
 *   id_lo, id_hi  uint32 low and high words of the uint64 particle id
 *       (unique, < 2^63).  Two arrays so that the mover, whose collision
 *       test draws from the id, reads 4 bytes per particle while every id
 *       of an instance is below 2^32 (its high words are then all zero).
 * An absorbed particle keeps its slot until the next sort, marked by
 * cell < 0 (PIC_FP32) or x < 0 (PIC_FP64).
 */
typedef struct {
    void *x[2];
    int32_t *cell[2];
    void *vx[2], *vy[2], *vz[2];
    uint32_t *id_lo[2], *id_hi[2];
    void *work;          /* device workspace of pic_sizes.work_bytes, 256-byte aligned */
} pic_buffers;

typedef struct {
    int64_t step;                 /* index of the next step */
    uint64_t next_id;
    uint32_t status;              /* PIC_ST_* bits */
    int32_t cur_set;              /* buffer set holding the particles */
    int64_t n_slots_used[PIC_MAX_SPECIES];  /* occupied slots (live + absorbed since last sort) */
    int64_t n_live[PIC_MAX_SPECIES];
    double ke[PIC_MAX_SPECIES];             /* sum 1/2 m w |V|^2 [J/m^2] */
    double mom[PIC_MAX_SPECIES][3];         /* sum m w V [kg/(m s)] */
    double field_energy;                    /* 1/2 eps0 sum_j E_j^2 V_j [J/m^2] */
    int64_t absorbed_total[PIC_MAX_SPECIES][2];  /* [left, right] wall */
    int64_t created_total[PIC_MAX_SPECIES];
    int64_t n_candidates, n_elastic, n_ionize, n_cx, n_over_cap, n_source;
    int64_t particle_steps;       /* particles pushed, summed over steps */
    int64_t n_excite;             /* excitation collisions */
    int64_t n_consumed;           /* neutral atoms consumed by ionisation */
    int64_t n_iz_untargeted;      /* ionisations whose cell had no atom left */
} pic_diag;

/* workspace regions readable by tests and tools (pic_region) */
typedef enum {
    PIC_R_DEPOSIT = 0,   /* uint64 [nsp][n_nodes]  fixed-point deposit S (2^32 per particle) */
    PIC_R_RHO = 1,       /* double [n_nodes]       charge density [C/m^3] */
    PIC_R_PHI = 2,       /* double [n_nodes]       potential [V] */
    PIC_R_EFIELD = 3,    /* double [n_nodes]       E_x [V/m] */
    PIC_R_ACC64 = 4,     /* double [nsp][n_nodes]  (q/m) E dt^2/dx, cells/step^2 */
    PIC_R_ACC32 = 5,     /* float  [nsp][n_nodes]  the same, rounded to FP32 */
    PIC_R_CELL_OFFSETS = 6, /* uint32 [nsp][n_nodes] first slot of each cell after the last sort */
    PIC_R_NODE_BASE = 7, /* int64 [n_inst+1]       first node of each instance */
    PIC_R_NEUTRAL_DENSITY = 8 /* double [n_nodes] density of the kinetic neutrals [m^-3] */
} pic_region_id;

typedef struct pic_ctx pic_ctx;

/* init flags */
#define PIC_INIT_NO_FIELD 0x1u   /* skip the initial deposit + field solve */
#define PIC_INIT_SORT     0x2u   /* sort the uploaded particles by cell first */
#define PIC_INIT_DEVICE   0x4u   /* draw the initial particles on the device (see pic_init) */

/* push flags */
#define PIC_PUSH_NO_DEPOSIT 0x1u /* do not deposit the new positions */

/*
 * pic_query_sizes -- host only, pure.  Validates n_inst configurations and
 * reports the buffer sizes.  seg_base (may be NULL) receives n_inst*nsp+1
 * slot offsets.  Returns PIC_OK, PIC_E_ARG or PIC_E_CONFIG.
 */
int pic_query_sizes(const pic_config *cfgs, int n_inst, pic_sizes *out, int64_t *seg_base);

/*
 * pic_init -- bind caller-owned buffers, convert the configuration to
 * cells/steps, write the per-segment tables, drop (and flag) uploaded
 * particles that are out of range or non-finite, optionally sort them by cell
 * (PIC_INIT_SORT; the particles then live in buffer set 1), and (unless
 * PIC_INIT_NO_FIELD) deposit them and solve the field so that the first
 * pic_push sees E at the initial positions.  stream is a hipStream_t (NULL =
 * the null stream).  Sec. 2: initialisation of grid and particles before the
 * cycle.  On error *out is NULL.
 *
 * PIC_INIT_DEVICE draws the n_init particles of every segment into buffer
 * set 0 instead of reading an upload.  Particle p of species k of instance i
 * gets id (n_init of the species before k) + p and two Philox4x32-10 blocks
 * keyed (seed_lo, seed_hi ^ i) with counter (id_lo, id_hi, 0xFFFFFFFF, b),
 * b = 0, 1 (step -1, before the first step):
 *   x = U(u0) nc, or (p + 1/2) nc / n_init with PIC_INIT_OPT_QUIET, or, with
 *       PIC_INIT_OPT_PAIR and the count of species 0, particle p of species
 *       0's final position; an electron species not so copied is displaced
 *       by (A/kk) sin(kk x), kk = 2 pi init_mode / nc, A = init_amp (wrapped
 *       when periodic); x is kept inside [0, nc).  U(u) = (u + 1/2) 2^-32.
 *   v = sqrt(T_init/m) dt/dx times standard normals from Box-Muller on
 *       (u1, u2) -> vx, vy and (u3, u'0) -> vz.
 * The FP32 form stores cell = floor(x) and f = x - cell rounded to float (an
 * f that rounds to 1 moves to the next cell, or stays below 1 in the last).
 * next_id must be at least the sum of n_init (PIC_E_CONFIG otherwise).
 */
int pic_init(const pic_config *cfgs, int n_inst, const pic_buffers *bufs, void *stream,
             unsigned flags, pic_ctx **out);

/*
 * pic_push -- the mover (Sec. 2 phase 5; moveb listing, Sec. 6): linear
 * gather of the grid acceleration at the in-cell offset, magnetised Boris
 * velocity update (half kick, rotation about B, half kick), position advance
 * x += vx, then plasma-wall interaction (absorbing walls, counted per wall,
 * or periodic re-entry).  Unless PIC_PUSH_NO_DEPOSIT, the new positions are
 * deposited (phase 1 of the next step) into the fixed-point arrays.  With
 * MCC on, every particle of a species with a collision process takes the
 * null-collision test; the selected ones are listed, with their velocities
 * and ids, for pic_mcc_collide.  Kinetic neutrals (q = 0) and every species
 * of a field-off instance move ballistically.
 */
int pic_push(pic_ctx *ctx, unsigned flags);

/*
 * pic_deposit -- phase 1 (Sec. 2, plasma density calculation) on its own:
 * adds every live particle's linear weights (F = 32 fixed point, 2^32 per
 * particle, order-independent) to PIC_R_DEPOSIT.
 */
int pic_deposit(pic_ctx *ctx);

/*
 * pic_field_solve -- phases 2 and 3 (Sec. 2, density smoother and field
 * solver): rho from the deposit, smoothed when smooth_passes > 0, the
 * tridiagonal Poisson solve in FP64 (Thomas recurrences), E = -grad(phi) and
 * the per-species grid acceleration; also the node density of a kinetic
 * neutral species (its deposit times its macro weight over the node volume).
 * A field-off instance gets E = phi = 0.  Consumes (clears) the deposit.
 */
int pic_field_solve(pic_ctx *ctx);

/*
 * pic_mcc_collide -- phase 4 (Sec. 2, collisions and plasma-wall
 * interaction): null-collision Monte Carlo for the particles listed by
 * pic_push (elastic e-n, excitation, charge exchange i-n, ionisation with
 * pair creation), the pair source refilling this step's ion wall loss, ids
 * of the created particles, and the close of the step (counters, step
 * index).  Must be called once per step after pic_push, also when MCC and
 * source are off.
 *
 * With a kinetic neutral species (the Table 1 case, Sec. 3.4) the electron
 * rates use the local atom density of the last field pass, gathered at the
 * electron with the mover's linear weights, and each ionisation consumes an
 * atom of its parent's cell: the events of a cell, in parent-id order, take
 * the live atoms of the cell (after this step's push) in the order of the
 * key (w0 << 32 | w1) of Philox block (id, step, 3) of the atom, ties by id;
 * the new ion is that atom (its position and velocity).  An event whose cell
 * has no atom left creates its ion at the parent with a Maxwellian draw at
 * T_n.  The atoms of a cell are found through the cell offsets of the last
 * pic_sort (a window of cells wide enough for the fastest atom since then),
 * or by a scan of the species when no sort has run.
 */
int pic_mcc_collide(pic_ctx *ctx);

/*
 * pic_sort -- "natural sorting" (Sec. 2, BIT1 data layout: particles grouped
 * by cell): counting sort of every segment by cell into the other buffer
 * set, dropping absorbed particles; writes PIC_R_CELL_OFFSETS.
 */
int pic_sort(pic_ctx *ctx);

/*
 * pic_diagnostics -- per-instance counts, kinetic energy, momentum, field
 * energy, wall losses, collision counts and the device status word.
 * Synchronises the stream (the only call that does).  out has n_inst
 * entries.  Returns PIC_OK, or the negative code of the most severe status
 * bit that is set (the diagnostics are filled in either way).
 */
int pic_diagnostics(pic_ctx *ctx, pic_diag *out, int n_inst);

/*
 * pic_step -- n_steps whole steps: pic_push, pic_mcc_collide,
 * pic_field_solve, and pic_sort every sort_every steps (counted from the
 * step index), enqueued back to back.
 */
int pic_step(pic_ctx *ctx, int n_steps, int sort_every);

/*
 * pic_step_graph -- the same n_steps whole steps as pic_step, with the same
 * results, replayed from a HIP graph: one sort period (sort_every steps with
 * the sort where pic_step puts it, or one step when sort_every is 0),
 * starting at the current step's phase of the cadence, is captured on a
 * stream the context owns, instantiated once (again when sort_every or the
 * phase changes) and launched on the context's stream once per whole period;
 * the remainder after the last whole period runs as in pic_step.  With
 * n_steps = 0 the graph for the current phase is captured and uploaded
 * without launching anything (so that a later call's first replay carries
 * no capture).  The captured work holds no memset and no host
 * synchronisation.  Returns PIC_E_DEVICE when capture or instantiation
 * fails.
 */
int pic_step_graph(pic_ctx *ctx, int n_steps, int sort_every);

/*
 * pic_autotune_sort -- choose the sort cadence by measurement ("natural
 * sorting", Sec. 2: how often to restore the order by cell).  For each of
 * the n_cand candidates (a cadence in steps, 0 = never) the particles are
 * sorted, then trial_steps whole steps run as in pic_step_graph and are
 * timed with HIP events; every candidate is timed in two interleaved
 * rounds, after one untimed warm-up trial, and rates[i] (may be NULL)
 * receives the better of its two rates in particle-steps per second; *best
 * receives the candidate with the highest.  The trials advance the
 * simulation by (2 n_cand + 1) trial_steps steps, like warm-up steps; make
 * trial_steps a multiple of every candidate so that each trial ends with a
 * sort.  Synchronises the stream.
 */
int pic_autotune_sort(pic_ctx *ctx, const int *cand, int n_cand, int trial_steps, int *best,
                      double *rates);

/*
 * pic_init_static -- pic_init for callers that cannot allocate device memory
 * (serving loops and harnesses that forbid hipMalloc): the workspace is not
 * a caller buffer but a static device array of the library, PIC_STATIC_WORK_MAX
 * bytes on each GPU it runs on, held until the process ends.  Same arguments,
 * checks, flags, work and results as pic_init, except:
 *   - bufs->work must be NULL (PIC_E_ARG otherwise); the particle buffers are
 *     the caller's, as for pic_init;
 *   - a configuration whose pic_sizes.work_bytes exceeds PIC_STATIC_WORK_MAX
 *     returns PIC_E_SCRATCH before any device work;
 *   - the array belongs to the device current at the call; while a context
 *     made by pic_init_static on that device is alive (until its
 *     pic_destroy), another pic_init_static there returns PIC_E_BUSY.  The
 *     array keeps the last context's contents; pic_init_static clears the
 *     part it uses, as pic_init clears its workspace;
 *   - no device or pinned host memory is allocated: the diagnostics are
 *     staged in the context (host memory), not in pinned memory.
 * The context is used with every other call like one from pic_init;
 * pic_region offsets are into the static array, which the caller cannot
 * address.  pic_step_graph on such a context still creates its capture
 * stream and graph.
 */
#define PIC_STATIC_WORK_MAX (64ull << 20)
int pic_init_static(const pic_config *cfgs, int n_inst, const pic_buffers *bufs, void *stream,
                    unsigned flags, pic_ctx **out);

/*
 * pic_set_mover -- the launch shape of the mover (Sec. 6 moveb loop; Sec.
 * 3.1-3.2 tune the matching OpenMP/OpenACC grain and team counts by hand):
 * chunks = 64-particle chunks a wave loads per pass over its part of a
 * 1024-particle tile (4: one pass; 2: two passes, fewer registers, more
 * waves per SIMD), blocks = persistent grid (0: pic_sizes.mover_blocks; at
 * most pic_sizes.mover_blocks_max).  Results are the same for every shape.
 * Host only; takes effect from the next step (call it between whole steps)
 * and drops the graph pic_step_graph captured.  PIC_E_ARG for other values.
 */
int pic_set_mover(pic_ctx *ctx, int chunks, int blocks);

/*
 * pic_autotune -- choose the mover's launch shape and the sort cadence by
 * measurement.  Each of the n_movers shapes (chunks[i], blocks[i]) runs
 * trial_steps whole steps at cadences[0] after a fresh sort; the fastest
 * (particle-steps per second, HIP events) is kept (*best_mover = its index)
 * and each of the n_cad cadences is then timed with it (*best_cadence = the
 * fastest value).  As in pic_autotune_sort, each set of candidates is timed
 * in two interleaved rounds after one untimed warm-up trial, and a
 * candidate's rate is the better of its two.  rates (may be NULL) receives
 * n_movers + n_cad rates.  The context is left on the best shape; the trials
 * advance the simulation like warm-up steps.  Synchronises the stream.
 */
int pic_autotune(pic_ctx *ctx, const int *chunks, const int *blocks, int n_movers,
                 const int *cadences, int n_cad, int trial_steps, int *best_mover,
                 int *best_cadence, double *rates);

/* pic_region -- byte offset (into pic_buffers.work) and element count of a
 * workspace region; host only. */
int pic_region(const pic_ctx *ctx, int region, uint64_t *byte_offset, int64_t *n_elems);

/* pic_destroy -- free the host context (no device memory is touched). */
int pic_destroy(pic_ctx *ctx);

/* pic_strerror -- static text for a pic_status code. */
const char *pic_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */
