// pic_internal.h -- device-side tables, workspace layout and launcher
// declarations of libpic.  Internal to the library (host code and kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"

namespace picx {

// ---------------------------------------------------------------------------
// launch geometry
// ---------------------------------------------------------------------------
constexpr int kBlock = 256;                 // threads per block of the particle kernels
constexpr int kWaves = kBlock / 64;         // wave64 per block
constexpr int kPer = 4;                     // 64-particle chunks per wave per tile
constexpr int kTile = kBlock * kPer;        // particles per tile (contiguous)
constexpr int kFieldR = 4;                  // nodes per thread in the field scans
constexpr int kFieldTile = kBlock * kFieldR;
constexpr int kSortR = 8;                   // bins per thread in the sort scan
constexpr int kSortTile = kBlock * kSortR;
constexpr int kDiagBlocks = 1024;           // blocks of the diagnostics reduction
constexpr int kEmitBlocks = 64;             // blocks of the emit/close-of-step kernel
constexpr int kEmitRankedBlocks = 512;      // blocks of the emit kernel that ranks its events (64 per block)
constexpr int kDiagVals = 6;                // live, sum v2, sum vx, vy, vz, (pad)
constexpr int kMaxPushBlocks = 256 * 8;     // candidate regions, and the largest grid of the particle kernels
constexpr int kCandQMin = 1024;             // least candidate entries per push block region
constexpr int kEvQMin = 32;                 // least ionisation-event slots per collide block
constexpr int kCntSegMax = 1024;           // segments counted per block in LDS (no atomics)
constexpr int kNCnt = 6;                    // candidates, elastic, ionisation, CX, over v_cap, excitation
constexpr int kRankJ = 64;                  // events compared per block pass of the rank kernel
constexpr int kRankBlocks = 512;            // grid of the rank kernel
constexpr int kTargetBlocks = 64;           // grid of the neutral-target kernel (a wave per event)
constexpr int kOvfCollideBlocks = 64;       // grid of the collide kernel for the overflow list only
constexpr uint32_t kNoIndex = 0xFFFFFFFFu;  // steps since the last sort: no sort yet

constexpr int32_t kDeadCell = -1;           // FP32 form: cell of an absorbed particle
constexpr double kDeadX = -1.0;             // FP64 form: position of an absorbed particle

// ---------------------------------------------------------------------------
// static per-segment constants (segment = instance x species)
// ---------------------------------------------------------------------------
struct SegConst {
    int64_t base;       // first slot
    int64_t tile0;      // first virtual particle tile of the segment
    int64_t gnode;      // first grid node of the instance
    int64_t node_stride;// G: distance between species rows of the [nsp][G] grid arrays
    uint32_t cap;       // slots
    int32_t inst, sp, kind;
    int32_t nstep;      // pushed on steps s with s mod nstep = 0, over nstep dt
    int32_t nc, bc, nsp, partner;   // partner: the other species' segment (MCC / source)
    // Boris rotation t = (q/m) B dt/2 (cos th, sin th, 0), s = 2t/(1+|t|^2)
    double tx, ty, sx, sy;
    float txf, tyf, sxf, syf;
    double ms;          // nstep as a double (kick, advance)
    float msf;
    // null-collision MCC (rates per step, speeds in cells/step)
    uint64_t T;         // candidate threshold floor(P 2^32), 0..2^32
    double nu_max;      // (n_n sig_all) dx vcap
    double C0, C1, C2;  // squares of the cumulative (n sig) dx: elastic, +excitation, +ionisation
    double crate;       // (n_n sig_iz) dx vcap: the constant-rate ionisation slot
    double vcap2, v2_iz, eps_iz, v2_ex;
    double vcap_hat;
    // kinetic neutrals: cross sections and dx (m) for the rates at the local density
    double sig_el, sig_ex, sig_iz, dxm, n_bound;
    int32_t kinetic;    // the instance has a kinetic neutral species (electron rates are local)
    int32_t rate_iz;    // PIC_XS_IZ_RATE
    int32_t force;      // 0: no field acts (q = 0 or the instance's field is off): no gather
    int32_t _pad1;
    double w;           // macro weight (real particles per macro-particle per unit area)
    double am, bm;      // m/(m+M), M/(m+M) (elastic, cold neutral of mass M)
    double sig_n;       // neutral Maxwellian sqrt(T_n/m_s) in cells/step (CX, new ions)
    double sig_src;     // source Maxwellian sqrt(T_src/m_s) in cells/step
    uint32_t key0, key1;
    // drawn initial state: particles, first id, Maxwellian sqrt(T/m) in cells/step
    int64_t n_init;
    uint64_t id0;
    double vth_init;
    // field / diagnostics
    double qw;          // q w
    double accC;        // (q/m) dt^2 / dx
    double mw, vs;      // m w, dx/dt
};

struct InstConst {
    int64_t gnode;      // first node
    int64_t ftile0;     // first field tile
    int32_t nc, bc, nsp, mcc_on, source_on, seg0, seg_e, seg_i;
    double dx, eps0, K; // K = dx^2 / eps0
    double init_amp;    // drawn initial state: perturbation amplitude, mode, PIC_INIT_OPT_*
    int32_t init_mode, init_opts;
    int32_t smooth_passes;
    int32_t field_off;  // no field solve (E = 0)
    int32_t seg_n;      // segment of the kinetic neutral species, or -1
    int32_t _pad;
};

// dynamic per-segment counters
struct SegDyn {
    uint32_t count;          // occupied slots (live + absorbed since the last sort)
    uint32_t live;
    uint32_t absorbed_step[2];
    uint32_t created_step;   // particles placed this step
    uint32_t consumed_step;  // kinetic neutrals consumed by ionisation this step
    unsigned long long absorbed_total[2];
    unsigned long long created_total;
    unsigned long long vmax_bits;  // kinetic neutrals: bits of max |vx| (double) at the last sort
};

// dynamic per-instance counters
struct InstDyn {
    long long step;
    unsigned long long next_id;
    uint32_t status;
    uint32_t wide_ids;  // some id of the instance may be >= 2^32 (the movers then read id_hi)
    // process counts of batches with more than kCntSegMax segments (otherwise per-block slots)
    unsigned long long n_candidates, n_elastic, n_ionize, n_cx, n_over_cap;
    unsigned long long n_source;
    unsigned long long particle_steps;
    unsigned long long n_consumed, n_iz_untargeted, n_excite;
};

// the movers' work queues: kUnitCtrs counters (grabs, waves done), one per
// 128-byte line
constexpr int kUnitCtrs = 32;
constexpr int kUnitCtrStride = 32;  // 32-bit words between counters

struct Globals {
    int32_t cur_set;
    uint32_t cand_ovf;       // candidates in the overflow list this step
    uint32_t ev_ovf;         // ionisation events in the overflow list this step
    uint32_t since_sort;     // steps closed since the last sort (kNoIndex: none yet)
    uint32_t ev_total;       // ionisation events this step (regions + overflow), from index_kernel
    uint32_t ev_in_regions;  // of which in the per-block regions
    uint32_t pad[2];
    // self-resetting single-pass scan (the sort): ticket counter, finish counter, generation
    uint32_t scan_ticket[4];
    uint32_t scan_finish[4];
    unsigned long long scan_gen[4];
    // the movers' unit counters (zero at set-up; each launch leaves them zero)
    unsigned int unit_ctr[kUnitCtrs * kUnitCtrStride];
};

enum ScanId { kScanSort = 2 };

// collision candidate listed by the mover: its slot, its velocity after the
// push (cells/step, exact in FP64 for both forms) and its id
struct Cand {
    uint32_t g;
    int32_t seg;            // its segment
    double vx, vy, vz;
    unsigned long long pid;
};

// ionisation event recorded by the collide kernel for the emit kernel
struct IzEvent {
    unsigned long long parent_id;
    uint32_t slot;          // parent slot (global)
    int32_t seg;            // parent segment
    int32_t inst;           // parent instance
    int32_t cell;           // parent cell (in-instance)
    double g2;              // speed of the secondary electron, cells/step
};

// an ionisation event in its instance's bucket (ranks of a batch)
struct RankEntry {
    unsigned long long pid;
    int32_t cell;
    uint32_t e;             // the event's index in the step's event list
};

// composite y -> A y + B of the maps of one tile of an affine (Thomas) sweep
struct AffineStatus {
    double A, B;
};

// a tile's backward composite phi_lo = A phi_above + B0 + B1 y, as a function
// of the value y of d' entering the tile from below
struct BackStatus {
    double A, B0, B1;
};

// a field node's forward-sweep terms: d' = d0 + h y for the d' y entering
// its tile from below
struct NodeSweep {
    double d0, h;
};

// ---------------------------------------------------------------------------
// workspace layout (byte offsets into pic_buffers.work)
// ---------------------------------------------------------------------------
struct Layout {
    uint64_t segc, instc, segd, instd, glob;
    uint64_t seg_tile0, seg_base, inst_ftile0, node_base;
    uint64_t S, rho, phi, E, dprime, acc64, acc32;
    uint64_t hist, cursor, offsets, seg_start;
    uint64_t fwd_status, bwd_status, sort_status, sweep, bpre;
    uint64_t fe_part;
    uint64_t cand, cand_n, ev, ev_n, ev_rank, cnt_slot;
    uint64_t nn, ev_crank, ev_target, ev_pre;
    uint64_t inst_ev, inst_fill, inst_start, rank_bucket;
    uint64_t diag_part, diag_out;
    uint64_t total;
    int64_t cand_ovf_cap, ev_ovf_cap;
    int64_t cand_q, ev_q;
    int64_t n_field_tiles, n_sort_tiles;
};

// every device pointer a kernel may need, passed by value
struct Dev {
    // particle sets
    void *x[2];
    int32_t *cell[2];
    void *vx[2], *vy[2], *vz[2];
    uint32_t *id_lo[2], *id_hi[2];   // low and high words of the particle ids
    // tables
    const SegConst *segc;
    const InstConst *instc;
    SegDyn *segd;
    InstDyn *instd;
    Globals *glob;
    const int64_t *seg_tile0;   // [n_seg+1]
    const int64_t *seg_base;    // [n_seg+1]
    const int64_t *inst_ftile0; // [n_inst+1]
    const int64_t *node_base;   // [n_inst+1]
    // grid
    unsigned long long *S;      // [nsp][G]
    double *rho, *phi, *E, *dprime;  // [G]
    double *acc64;              // [nsp][G]
    float *acc32;               // [nsp][G]
    uint32_t *hist, *cursor, *offsets;  // [nsp][G]
    unsigned long long *seg_start;      // [n_seg] first raw sort position of each segment
    AffineStatus *fwd_status;
    BackStatus *bwd_status;
    NodeSweep *sweep;   // [n_field_tiles * kFieldTile] per node, tile by tile
    BackStatus *bpre;   // [n_field_tiles * kBlock] backward maps above each thread's nodes
    unsigned long long *sort_status;
    double *fe_part;
    Cand *cand;                 // [n_regions][cand_q] per-block regions, then the overflow list
    uint32_t *cand_n;           // [n_regions][kWaves] candidates in each wave's part of a region
    IzEvent *ev;                // [n_regions][ev_q] per-block regions, then the overflow list
    uint32_t *ev_n;             // [n_regions] events in each region (the first n_push_blocks in use)
    uint32_t *ev_rank;          // [events] rank of each event among its instance's (by parent id)
    uint32_t *ev_crank;         // [events] rank among the events of its instance and cell
    long long *ev_target;       // [events] slot of the atom an event consumes, or -1
    double *nn;                 // [G] density of the kinetic neutrals [m^-3]
    uint32_t *ev_pre;           // [n_push_blocks+1] first event of each region (index_kernel)
    // ranks of a batch: events per instance, fill counters, bucket starts, buckets
    uint32_t *inst_ev, *inst_fill, *inst_start;   // [n_inst], [n_inst], [n_inst+1]
    RankEntry *rank_bucket;                        // [events]
    unsigned long long *cnt_slot;  // [n_regions][n_seg][kNCnt] process counts per collide block
    double *diag_part;
    pic_diag *diag_out;
    // sizes
    int64_t n_slots, n_tiles, G, cand_ovf_cap, ev_ovf_cap;
    int64_t n_field_tiles, n_sort_tiles;
    int32_t n_seg, n_inst, nsp, precision;
    int32_t n_push_blocks;      // grid of the movers and the collide kernel (regions in use)
    int32_t n_regions;          // candidate / event regions of the layout (>= n_push_blocks)
    int32_t kinetic_any;        // some instance has a kinetic neutral species (with MCC on)
    int32_t cand_q, ev_q;       // entries per block region of the candidate and event lists
    int32_t field_all_off;      // no instance solves the field
    int32_t late_flush;         // the FP32 mover flushes its deposit window after the next pass's loads
};

// a particle's id from its two words
__device__ __forceinline__ unsigned long long load_id(const Dev &d, int set, int64_t g)
{
    return (unsigned long long)d.id_lo[set][g] | ((unsigned long long)d.id_hi[set][g] << 32);
}

__device__ __forceinline__ void store_id(const Dev &d, int set, int64_t g, unsigned long long id)
{
    d.id_lo[set][g] = (uint32_t)id;
    d.id_hi[set][g] = (uint32_t)(id >> 32);
}

// ---------------------------------------------------------------------------
// launchers (each enqueues on `st`; return hipError_t)
// ---------------------------------------------------------------------------
hipError_t launch_init_state(const Dev &d, hipStream_t st, const uint32_t *n_init_dev);
// draws the initial particles of every segment into buffer set 0
hipError_t launch_init_device(const Dev &d, hipStream_t st);
// mcc: test every particle and list the candidates (pic_mcc_collide collides them)
// subcycled: some species has nstep > 1 (its deposit between pushes is launched too)
// chunks: 64-particle chunks a mover wave loads per pass (kPer, or kPer / 2
// in two passes per tile)
// collide (with mcc): each mover block then collides the candidates of its
// own region (the shared overflow list is left to launch_collide)
hipError_t launch_push(const Dev &d, hipStream_t st, bool deposit, bool mcc, bool subcycled, int chunks,
                       bool collide);
hipError_t launch_deposit(const Dev &d, hipStream_t st);
// smooth: the most density-smoother passes of any instance; close_mode >= 0:
// the first launch also closes the step (close_step's mode; no instance may
// have a periodic background, whose rho reads the counts the close updates)
hipError_t launch_field(const Dev &d, hipStream_t st, int smooth, int close_mode = -1);
// overflow_only: after movers that collided their own regions (launch_push
// with collide), only the shared overflow list is left
hipError_t launch_collide(const Dev &d, hipStream_t st, bool overflow_only);
// ionisation and source pairs (when `pairs`), then the close of the step
// (`events`: collisions ran this step); with `deferred_close`, the close is
// not launched and its mode is stored there, for launch_field
hipError_t launch_emit(const Dev &d, hipStream_t st, bool pairs, bool events, int *deferred_close = nullptr);
hipError_t launch_sort(const Dev &d, hipStream_t st);
hipError_t launch_diag(const Dev &d, hipStream_t st);

int push_grid(const Dev &d);

// ---------------------------------------------------------------------------
// host side: context set-up shared by pic_init and pic_init_static
// ---------------------------------------------------------------------------
// workspace bytes of a configuration (0 and *rc < 0 when it is invalid)
uint64_t work_bytes_of(const pic_config *cfgs, int n_inst, int *rc);
// pic_init with the workspace at W; pinned_diag: stage the diagnostics in
// pinned host memory, else in the context
int init_context(const pic_config *cfgs, int n_inst, const pic_buffers *bufs, void *W,
                 void *stream, unsigned flags, bool pinned_diag, pic_ctx **out);
// the context holds the static workspace of `device` (released by pic_destroy)
void mark_static(pic_ctx *c, int device);
void static_release(int device);

}  // namespace picx
