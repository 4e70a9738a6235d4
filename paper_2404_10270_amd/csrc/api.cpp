// api.cpp -- host side of libpic: validation, buffer sizes, workspace layout,
// unit conversion into cells and steps, and the per-phase launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "pic.h"
#include "pic_internal.h"

using namespace picx;

struct pic_ctx {
    std::vector<pic_config> cfg;
    int n_inst = 0, nsp = 0, precision = 0;
    bool mcc_any = false, src_any = false;
    int max_smooth = 0;       // most smoother passes of any instance
    bool sub_any = false;     // some species is subcycled (nstep > 1)
    bool periodic_any = false;  // some instance is periodic (its rho reads the live counts)
    Layout L{};
    Dev d{};
    hipStream_t st = nullptr;
    int64_t host_steps = 0;   // steps enqueued since init
    pic_diag *host_diag = nullptr;  // staging for pic_diagnostics: pinned (pic_init) ...
    bool host_diag_pinned = false;
    std::vector<pic_diag> diag_stage;  // ... or held here (pic_init_static)
    int static_dev = -1;            // device whose static workspace this context holds
    int chunks = kPer;              // mover chunks per wave and pass (pic_set_mover)
    int default_blocks = 1;         // the layout's default mover grid
    // pic_step_graph: one sort period captured on a stream of its own
    hipStream_t cap_st = nullptr;
    hipGraphExec_t gexec = nullptr;
    int g_period = 0, g_sort = -1, g_phase = 0;
};

namespace {

constexpr uint64_t kAlign = 256;
constexpr int kMaxInst = 4096;
constexpr int64_t kMaxSlots = 0xFFFFFFF0ll;  // slots are addressed with uint32

uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }
bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

int find_kind(const pic_config &c, int kind)
{
    for (int k = 0; k < c.nsp; ++k)
        if (c.sp[k].kind == kind) return k;
    return -1;
}

int count_kind(const pic_config &c, int kind)
{
    int n = 0;
    for (int k = 0; k < c.nsp; ++k) n += c.sp[k].kind == kind;
    return n;
}

int validate(const pic_config *cfgs, int n_inst)
{
    if (!cfgs || n_inst < 1 || n_inst > kMaxInst) return PIC_E_ARG;
    const int nsp = cfgs[0].nsp, prec = cfgs[0].precision;
    if (nsp < 1 || nsp > PIC_MAX_SPECIES) return PIC_E_CONFIG;
    if (prec != PIC_FP32 && prec != PIC_FP64) return PIC_E_CONFIG;
    for (int i = 0; i < n_inst; ++i) {
        const pic_config &c = cfgs[i];
        if (c.nsp != nsp || c.precision != prec) return PIC_E_CONFIG;
        if (c.nc < 2 || c.nc > (1 << 26)) return PIC_E_CONFIG;
        if (c.bc != PIC_BC_PERIODIC && c.bc != PIC_BC_ABSORB) return PIC_E_CONFIG;
        if (!finite_pos(c.dx) || !finite_pos(c.dt) || !finite_pos(c.eps0)) return PIC_E_CONFIG;
        if (!finite_nonneg(c.B0) || !std::isfinite(c.theta)) return PIC_E_CONFIG;
        if (c.next_id >= (1ull << 62) || c.step0 < 0) return PIC_E_CONFIG;
        if (c.smooth_passes < 0 || c.smooth_passes > 64) return PIC_E_CONFIG;
        if (c.field_off != 0 && c.field_off != 1) return PIC_E_CONFIG;
        if (c.xs_flags & ~PIC_XS_IZ_RATE) return PIC_E_CONFIG;
        if (count_kind(c, PIC_KIND_NEUTRAL) > 1) return PIC_E_CONFIG;
        for (int k = 0; k < nsp; ++k) {
            const pic_species &s = c.sp[k];
            if (!std::isfinite(s.q) || !finite_pos(s.m) || !finite_pos(s.w)) return PIC_E_CONFIG;
            if (s.kind != PIC_KIND_ELECTRON && s.kind != PIC_KIND_ION && s.kind != PIC_KIND_NEUTRAL)
                return PIC_E_CONFIG;
            if (s.kind == PIC_KIND_NEUTRAL && s.q != 0.0) return PIC_E_CONFIG;
            if (s.nstep < 0 || s.nstep > 1000000) return PIC_E_CONFIG;
            if (s.capacity < 1 || s.n_init < 0 || s.n_init > s.capacity) return PIC_E_CONFIG;
            if (s.capacity > kMaxSlots) return PIC_E_CONFIG;
        }
        // collisions and the source: one electron and one ion species, and
        // at most one kinetic neutral species besides
        if (c.mcc_on || c.source_on) {
            const int nn = count_kind(c, PIC_KIND_NEUTRAL);
            if (count_kind(c, PIC_KIND_ELECTRON) != 1 || count_kind(c, PIC_KIND_ION) != 1 ||
                nsp != 2 + nn)
                return PIC_E_CONFIG;
        }
        if (c.mcc_on) {
            if (!finite_nonneg(c.n_n) || !finite_nonneg(c.T_n) || !finite_nonneg(c.sig_el) ||
                !finite_nonneg(c.sig_iz) || !finite_nonneg(c.E_iz) || !finite_nonneg(c.sig_cx) ||
                !finite_nonneg(c.sig_ex) || !finite_nonneg(c.E_ex))
                return PIC_E_CONFIG;
            // no ion-neutral process with kinetic neutrals (the atom would have to change too)
            if (find_kind(c, PIC_KIND_NEUTRAL) >= 0 && c.sig_cx != 0.0) return PIC_E_CONFIG;
            for (int k = 0; k < nsp; ++k)
                if (c.sp[k].kind != PIC_KIND_NEUTRAL && !finite_pos(c.sp[k].v_cap)) return PIC_E_CONFIG;
        }
        if (c.source_on)
            for (int k = 0; k < nsp; ++k)
                if (!finite_nonneg(c.sp[k].T_src)) return PIC_E_CONFIG;
    }
    return PIC_OK;
}

// the configuration of a drawn initial state (PIC_INIT_DEVICE)
int validate_device_init(const pic_config *cfgs, int n_inst)
{
    for (int i = 0; i < n_inst; ++i) {
        const pic_config &c = cfgs[i];
        uint64_t total = 0;
        for (int k = 0; k < c.nsp; ++k) {
            if (!finite_nonneg(c.sp[k].T_init)) return PIC_E_CONFIG;
            total += (uint64_t)c.sp[k].n_init;
        }
        if (c.next_id < total) return PIC_E_CONFIG;
        if (!std::isfinite(c.init_amp)) return PIC_E_CONFIG;
        if (c.init_amp != 0.0 && c.init_mode == 0) return PIC_E_CONFIG;
        if (c.init_opts & ~(PIC_INIT_OPT_QUIET | PIC_INIT_OPT_PAIR)) return PIC_E_CONFIG;
    }
    return PIC_OK;
}

// slots of a segment, rounded to a multiple of 64 so that every segment
// starts on a 256-byte boundary of each array
int64_t seg_slots(const pic_species &s) { return (int64_t)align_up((uint64_t)s.capacity, 64); }

// candidate-list capacity: mean plus a wide margin of the binomial count
int64_t cand_capacity(const pic_config *cfgs, int n_inst, const std::vector<double> &P)
{
    double tot = 0.0;
    int q = 0;
    for (int i = 0; i < n_inst; ++i)
        for (int k = 0; k < cfgs[i].nsp; ++k, ++q) {
            const double cap = (double)cfgs[i].sp[k].capacity;
            const double mu = cap * P[q];
            tot += std::fmin(cap, mu + 10.0 * std::sqrt(mu + 1.0) + 256.0);
        }
    return (int64_t)align_up((uint64_t)tot + 1024, 256);
}

// Conversion of the configuration into cells and steps (one per segment).
// The candidate threshold is floor(P 2^32) with P = 1 - exp(-nu_max dt).
void seg_constants(const pic_config &c, int inst, int k, SegConst &s)
{
    const pic_species &sp = c.sp[k];
    const double dx = c.dx, dt = c.dt;
    s.inst = inst;
    s.sp = k;
    s.kind = sp.kind;
    s.nstep = sp.nstep > 1 ? sp.nstep : 1;
    s.ms = (double)s.nstep;
    s.msf = (float)s.nstep;
    s.nc = c.nc;
    s.bc = c.bc;
    s.nsp = c.nsp;
    s.partner = -1;
    const double tm = (sp.q / sp.m) * c.B0 * (0.5 * (dt * s.ms));
    s.tx = tm * std::cos(c.theta);
    s.ty = tm * std::sin(c.theta);
    const double den = 1.0 + (s.tx * s.tx + s.ty * s.ty);
    s.sx = 2.0 * s.tx / den;
    s.sy = 2.0 * s.ty / den;
    s.txf = (float)s.tx;
    s.tyf = (float)s.ty;
    s.sxf = (float)s.sx;
    s.syf = (float)s.sy;
    s.qw = sp.q * sp.w;
    s.accC = (sp.q / sp.m) * (dt * dt / dx);
    s.mw = sp.m * sp.w;
    s.vs = dx / dt;
    s.key0 = (uint32_t)c.seed;
    s.key1 = (uint32_t)(c.seed >> 32) ^ (uint32_t)inst;
    s.w = sp.w;
    s.force = (sp.q != 0.0 && !c.field_off) ? 1 : 0;  // else no gather: the acceleration is 0
    s.T = 0;
    s.nu_max = s.C0 = s.C1 = s.C2 = s.crate = 0.0;
    s.vcap2 = s.v2_iz = s.eps_iz = s.v2_ex = s.vcap_hat = s.am = s.bm = s.sig_n = 0.0;
    s.sig_el = s.sig_ex = s.sig_iz = 0.0;
    s.dxm = dx;
    s.n_bound = c.n_n;
    s.kinetic = s.rate_iz = 0;
    s.sig_src = 0.0;
    if (c.source_on) s.sig_src = std::sqrt(sp.T_src / sp.m) * (dt / dx);
    if (c.mcc_on) {
        const int ki = find_kind(c, PIC_KIND_ION), kn = find_kind(c, PIC_KIND_NEUTRAL);
        const double M = kn >= 0 ? c.sp[kn].m : c.sp[ki].m;  // neutral (elastic target) mass
        // cumulative (n sigma) dx of the processes, in the bound's density n_n
        double sig = 0.0, c0 = 0.0, c1 = 0.0, c2 = 0.0;
        if (sp.kind == PIC_KIND_ELECTRON) {
            sig = (c.sig_el + c.sig_ex) + c.sig_iz;
            c0 = (c.n_n * c.sig_el) * dx;
            c1 = (c.n_n * (c.sig_el + c.sig_ex)) * dx;
            c2 = (c.n_n * ((c.sig_el + c.sig_ex) + c.sig_iz)) * dx;
        } else if (sp.kind == PIC_KIND_ION) {
            sig = c.sig_cx;
            c0 = (c.n_n * c.sig_cx) * dx;
            c1 = c2 = c0;
        }
        const double vcap_hat = sp.v_cap * (dt / dx);
        const double nu_max_T = c.n_n * sig * dx * vcap_hat;
        const double P = -std::expm1(-(nu_max_T * s.ms));  // per push of nstep steps
        double T = std::floor(std::ldexp(P, 32));
        if (T > 4294967296.0) T = 4294967296.0;
        s.T = (uint64_t)T;
        s.nu_max = nu_max_T;
        s.C0 = c0 * c0;
        s.C1 = c1 * c1;
        s.C2 = c2 * c2;
        s.crate = ((c.n_n * c.sig_iz) * dx) * vcap_hat;
        s.vcap2 = vcap_hat * vcap_hat;
        s.vcap_hat = vcap_hat;
        s.v2_iz = (2.0 * c.E_iz / sp.m) * ((dt / dx) * (dt / dx));
        s.eps_iz = 0.5 * s.v2_iz;
        s.v2_ex = (2.0 * c.E_ex / sp.m) * ((dt / dx) * (dt / dx));
        s.am = sp.m / (sp.m + M);
        s.bm = M / (sp.m + M);
        s.sig_n = std::sqrt(c.T_n / sp.m) * (dt / dx);
        s.sig_el = c.sig_el;
        s.sig_ex = c.sig_ex;
        s.sig_iz = c.sig_iz;
        s.kinetic = (kn >= 0 && sp.kind == PIC_KIND_ELECTRON) ? 1 : 0;
        s.rate_iz = (c.xs_flags & PIC_XS_IZ_RATE) ? 1 : 0;
    }
}

double candidate_probability(const pic_config &c, int k)
{
    if (!c.mcc_on) return 0.0;
    SegConst s{};
    seg_constants(c, 0, k, s);
    return (double)s.T / 4294967296.0;
}

struct Plan {
    int64_t n_slots = 0, n_tiles = 0, G = 0, n_field_tiles = 0, n_sort_tiles = 0;
    int n_push_blocks = 1, n_regions = 1;
    std::vector<int64_t> seg_base, seg_tile0, node_base, inst_ftile0;
    Layout L{};
};

int plan(const pic_config *cfgs, int n_inst, Plan &p)
{
    const int nsp = cfgs[0].nsp;
    const int n_seg = n_inst * nsp;
    p.seg_base.assign(n_seg + 1, 0);
    p.seg_tile0.assign(n_seg + 1, 0);
    p.node_base.assign(n_inst + 1, 0);
    p.inst_ftile0.assign(n_inst + 1, 0);
    std::vector<double> P(n_seg, 0.0);
    for (int i = 0; i < n_inst; ++i) {
        for (int k = 0; k < nsp; ++k) {
            const int s = i * nsp + k;
            const int64_t n = seg_slots(cfgs[i].sp[k]);
            p.seg_base[s + 1] = p.seg_base[s] + n;
            p.seg_tile0[s + 1] = p.seg_tile0[s] + (n + kTile - 1) / kTile;
            P[s] = candidate_probability(cfgs[i], k);
        }
        const int64_t nodes = (int64_t)cfgs[i].nc + 1;
        p.node_base[i + 1] = p.node_base[i] + nodes;
        p.inst_ftile0[i + 1] = p.inst_ftile0[i] + (nodes + kFieldTile - 1) / kFieldTile;
    }
    p.n_slots = p.seg_base[n_seg];
    if (p.n_slots > kMaxSlots) return PIC_E_CONFIG;
    p.n_tiles = p.seg_tile0[n_seg];
    p.G = p.node_base[n_inst];
    p.n_field_tiles = p.inst_ftile0[n_inst];
    const int64_t nbins = (int64_t)nsp * p.G;
    p.n_sort_tiles = (nbins + kSortTile - 1) / kSortTile;

    Layout &L = p.L;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align_up(off + (bytes ? bytes : 1), kAlign);
        return o;
    };
    L.segc = take(sizeof(SegConst) * n_seg);
    L.instc = take(sizeof(InstConst) * n_inst);
    L.segd = take(sizeof(SegDyn) * n_seg);
    L.instd = take(sizeof(InstDyn) * n_inst);
    L.glob = take(sizeof(Globals));
    L.seg_tile0 = take(sizeof(int64_t) * (n_seg + 1));
    L.seg_base = take(sizeof(int64_t) * (n_seg + 1));
    L.inst_ftile0 = take(sizeof(int64_t) * (n_inst + 1));
    L.node_base = take(sizeof(int64_t) * (n_inst + 1));
    L.S = take(sizeof(uint64_t) * nbins);
    L.rho = take(sizeof(double) * p.G);
    L.phi = take(sizeof(double) * p.G);
    L.E = take(sizeof(double) * p.G);
    L.dprime = take(sizeof(double) * p.G);
    L.acc64 = take(sizeof(double) * nbins);
    L.acc32 = take(sizeof(float) * nbins);
    L.hist = take(sizeof(uint32_t) * nbins);
    L.cursor = take(sizeof(uint32_t) * nbins);
    L.offsets = take(sizeof(uint32_t) * nbins);
    L.seg_start = take(sizeof(uint64_t) * n_seg);
    L.fwd_status = take(sizeof(AffineStatus) * p.n_field_tiles);
    L.bwd_status = take(sizeof(BackStatus) * p.n_field_tiles);
    L.sweep = take(sizeof(NodeSweep) * p.n_field_tiles * kFieldTile);
    L.bpre = take(sizeof(BackStatus) * p.n_field_tiles * kBlock);
    L.sort_status = take(sizeof(uint64_t) * p.n_sort_tiles);
    L.fe_part = take(sizeof(double) * p.n_field_tiles);
    // candidates: one region per push block, sized so that a block holds
    // 1.25 times its share of the candidates of a full capacity (the shared
    // overflow list, whose appends contend on one counter, stays rare), then
    // an overflow list sized for the expected total (mean + 10 sigma).  The
    // persistent grid is one residency of the mover on 256 CUs: 4 blocks per
    // CU (both movers fit 4 waves per SIMD: 128 VGPRs or fewer).  A partial
    // second residency leaves the mover's last blocks running alone, and
    // fewer regions make the collide kernel (a block per region) and the
    // event index over the regions cheaper.  (pic_set_mover can run the
    // movers on up to twice that grid: the layout holds regions for it, each
    // sized for the default grid)
    const int max_blocks = 256 * 4;
    p.n_push_blocks = (int)std::min<int64_t>(std::max<int64_t>(p.n_tiles, 1), max_blocks);
    p.n_regions = (int)std::min<int64_t>(std::max<int64_t>(p.n_tiles, 1), 2 * max_blocks);
    L.cand_ovf_cap = cand_capacity(cfgs, n_inst, P);
    L.ev_ovf_cap = L.cand_ovf_cap;
    double expect = 0.0;
    for (int s = 0; s < n_seg; ++s) {
        const pic_config &cf = cfgs[s / nsp];
        expect += (double)cf.sp[s % nsp].capacity * P[s];
    }
    L.cand_q = std::max<int64_t>(kCandQMin,
                                 (int64_t)align_up((uint64_t)(1.25 * expect / p.n_push_blocks) + 64, 64));
    L.ev_q = std::max<int64_t>(kEvQMin, L.cand_q / 16);
    L.cand = take(sizeof(Cand) * ((uint64_t)p.n_regions * L.cand_q + L.cand_ovf_cap));
    L.cand_n = take(sizeof(uint32_t) * p.n_regions * kWaves);
    L.ev = take(sizeof(IzEvent) * ((uint64_t)p.n_regions * L.ev_q + L.ev_ovf_cap));
    L.ev_n = take(sizeof(uint32_t) * p.n_regions);
    L.ev_rank = take(sizeof(uint32_t) * ((uint64_t)p.n_regions * L.ev_q + L.ev_ovf_cap));
    L.ev_crank = take(sizeof(uint32_t) * ((uint64_t)p.n_regions * L.ev_q + L.ev_ovf_cap));
    L.ev_target = take(sizeof(long long) * ((uint64_t)p.n_regions * L.ev_q + L.ev_ovf_cap));
    L.nn = take(sizeof(double) * p.G);
    L.ev_pre = take(sizeof(uint32_t) * ((uint64_t)p.n_regions + 1));
    L.inst_ev = take(sizeof(uint32_t) * n_inst);
    L.inst_fill = take(sizeof(uint32_t) * n_inst);
    L.inst_start = take(sizeof(uint32_t) * (n_inst + 1));
    L.rank_bucket = take(sizeof(RankEntry) * ((uint64_t)p.n_regions * L.ev_q + L.ev_ovf_cap));
    L.cnt_slot = take(sizeof(unsigned long long) * (uint64_t)p.n_regions *
                      (n_seg <= kCntSegMax ? n_seg : 0) * kNCnt);
    L.diag_part = take(sizeof(double) * (uint64_t)kDiagBlocks * n_seg * kDiagVals);
    L.diag_out = take(sizeof(pic_diag) * n_inst);
    L.total = off;
    L.n_field_tiles = p.n_field_tiles;
    L.n_sort_tiles = p.n_sort_tiles;
    return PIC_OK;
}

bool aligned(const void *p) { return p && ((uintptr_t)p % kAlign) == 0; }

template <typename T>
T *at(void *work, uint64_t off)
{
    return (T *)((char *)work + off);
}

int status_code(uint32_t st)
{
    if (st & (PIC_ST_NONFINITE)) return PIC_E_NONFINITE;
    if (st & PIC_ST_CFL) return PIC_E_CFL;
    if (st & (PIC_ST_CAPACITY | PIC_ST_CANDIDATES | PIC_ST_BAD_INIT)) return PIC_E_CAPACITY;
    if (st & PIC_ST_INTERNAL) return PIC_E_STATE;
    return PIC_OK;
}

}  // namespace

extern "C" {

int pic_query_sizes(const pic_config *cfgs, int n_inst, pic_sizes *out, int64_t *seg_base)
{
    if (!out) return PIC_E_ARG;
    const int rc = validate(cfgs, n_inst);
    if (rc) return rc;
    Plan p;
    const int rc2 = plan(cfgs, n_inst, p);
    if (rc2) return rc2;
    out->n_slots = p.n_slots;
    out->n_segments = (int64_t)n_inst * cfgs[0].nsp;
    out->n_nodes = p.G;
    out->work_bytes = p.L.total;
    out->x_elem_bytes = cfgs[0].precision == PIC_FP64 ? 8 : 4;
    out->v_elem_bytes = out->x_elem_bytes;
    out->mover_blocks = p.n_push_blocks;
    out->mover_blocks_max = p.n_regions;
    if (seg_base)
        for (size_t s = 0; s < p.seg_base.size(); ++s) seg_base[s] = p.seg_base[s];
    return PIC_OK;
}

}  // extern "C"

namespace picx {

uint64_t work_bytes_of(const pic_config *cfgs, int n_inst, int *rc)
{
    *rc = validate(cfgs, n_inst);
    if (*rc) return 0;
    Plan p;
    *rc = plan(cfgs, n_inst, p);
    return *rc ? 0 : p.L.total;
}

// pic_init with the workspace at W (bufs->work is not read).  pinned_diag:
// stage the diagnostics in pinned host memory (pic_init) or in the context
// itself (pic_init_static, which allocates no device or pinned memory).
int init_context(const pic_config *cfgs, int n_inst, const pic_buffers *bufs, void *W,
                 void *stream, unsigned flags, bool pinned_diag, pic_ctx **out)
{
    if (!out) return PIC_E_ARG;
    *out = nullptr;
    if (!bufs) return PIC_E_ARG;
    const int rc = validate(cfgs, n_inst);
    if (rc) return rc;
    if (flags & PIC_INIT_DEVICE) {
        const int rc1 = validate_device_init(cfgs, n_inst);
        if (rc1) return rc1;
    }
    Plan p;
    const int rc2 = plan(cfgs, n_inst, p);
    if (rc2) return rc2;
    const bool f64 = cfgs[0].precision == PIC_FP64;
    for (int b = 0; b < 2; ++b) {
        if (!aligned(bufs->x[b]) || !aligned(bufs->vx[b]) || !aligned(bufs->vy[b]) ||
            !aligned(bufs->vz[b]) || !aligned(bufs->id_lo[b]) || !aligned(bufs->id_hi[b]))
            return PIC_E_ARG;
        if (!f64 && !aligned(bufs->cell[b])) return PIC_E_ARG;
    }
    if (!aligned(W)) return PIC_E_ARG;

    pic_ctx *c = new (std::nothrow) pic_ctx();
    if (!c) return PIC_E_ARG;
    c->cfg.assign(cfgs, cfgs + n_inst);
    c->n_inst = n_inst;
    c->nsp = cfgs[0].nsp;
    c->precision = cfgs[0].precision;
    c->st = (hipStream_t)stream;
    c->L = p.L;
    for (int i = 0; i < n_inst; ++i) {
        c->mcc_any = c->mcc_any || cfgs[i].mcc_on;
        c->src_any = c->src_any || cfgs[i].source_on;
        c->periodic_any = c->periodic_any || cfgs[i].bc == PIC_BC_PERIODIC;
        for (int k = 0; k < cfgs[i].nsp; ++k) c->sub_any = c->sub_any || cfgs[i].sp[k].nstep > 1;
    }

    const int nsp = c->nsp, n_seg = n_inst * nsp;
    std::vector<SegConst> segc(n_seg);
    std::vector<InstConst> instc(n_inst);
    std::vector<SegDyn> segd(n_seg);
    std::vector<InstDyn> instd(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const pic_config &cf = cfgs[i];
        InstConst &ic = instc[i];
        std::memset(&ic, 0, sizeof(ic));
        ic.gnode = p.node_base[i];
        ic.ftile0 = p.inst_ftile0[i];
        ic.nc = cf.nc;
        ic.bc = cf.bc;
        ic.nsp = nsp;
        ic.mcc_on = cf.mcc_on;
        ic.source_on = cf.source_on;
        ic.seg0 = i * nsp;
        const int ke = find_kind(cf, PIC_KIND_ELECTRON), ki = find_kind(cf, PIC_KIND_ION);
        ic.seg_e = (cf.mcc_on || cf.source_on) && ke >= 0 ? i * nsp + ke : -1;
        ic.seg_i = (cf.mcc_on || cf.source_on) && ki >= 0 ? i * nsp + ki : -1;
        ic.dx = cf.dx;
        ic.eps0 = cf.eps0;
        ic.K = cf.dx * cf.dx / cf.eps0;
        ic.init_amp = cf.init_amp;
        ic.init_mode = cf.init_mode;
        ic.init_opts = (int32_t)cf.init_opts;
        ic.smooth_passes = cf.smooth_passes;
        ic.field_off = cf.field_off;
        const int kn = find_kind(cf, PIC_KIND_NEUTRAL);
        ic.seg_n = kn >= 0 ? i * nsp + kn : -1;
        if (!cf.field_off && cf.smooth_passes > c->max_smooth) c->max_smooth = cf.smooth_passes;
        int64_t id0 = 0;
        for (int k = 0; k < nsp; ++k) {
            const int s = i * nsp + k;
            SegConst &sc = segc[s];
            std::memset(&sc, 0, sizeof(sc));
            seg_constants(cf, i, k, sc);
            sc.base = p.seg_base[s];
            sc.tile0 = p.seg_tile0[s];
            sc.gnode = p.node_base[i];
            sc.node_stride = p.G;
            sc.cap = (uint32_t)cf.sp[k].capacity;
            sc.n_init = cf.sp[k].n_init;
            sc.id0 = (uint64_t)id0;
            id0 += cf.sp[k].n_init;
            sc.vth_init = cf.sp[k].T_init > 0.0 ? std::sqrt(cf.sp[k].T_init / cf.sp[k].m) * cf.dt / cf.dx
                                                : 0.0;
            if (ic.seg_e >= 0 && ic.seg_i >= 0) {
                if (s == ic.seg_e) sc.partner = ic.seg_i;
                if (s == ic.seg_i) sc.partner = ic.seg_e;
            }
            SegDyn &sd = segd[s];
            std::memset(&sd, 0, sizeof(sd));
            sd.count = (uint32_t)cf.sp[k].n_init;
            sd.live = (uint32_t)cf.sp[k].n_init;
        }
        InstDyn &id = instd[i];
        std::memset(&id, 0, sizeof(id));
        id.step = cf.step0;
        id.next_id = cf.next_id;
        id.wide_ids = cf.next_id > (1ull << 32) ? 1u : 0u;  // (uploaded ids are checked by the device)
    }
    Globals g;
    std::memset(&g, 0, sizeof(g));
    g.cur_set = 0;
    g.since_sort = kNoIndex;  // no cell offsets yet
    for (int q = 0; q < 4; ++q) g.scan_gen[q] = 1;

    Dev &d = c->d;
    for (int b = 0; b < 2; ++b) {
        d.x[b] = bufs->x[b];
        d.cell[b] = bufs->cell[b];
        d.vx[b] = bufs->vx[b];
        d.vy[b] = bufs->vy[b];
        d.vz[b] = bufs->vz[b];
        d.id_lo[b] = bufs->id_lo[b];
        d.id_hi[b] = bufs->id_hi[b];
    }
    const Layout &L = c->L;
    d.segc = at<SegConst>(W, L.segc);
    d.instc = at<InstConst>(W, L.instc);
    d.segd = at<SegDyn>(W, L.segd);
    d.instd = at<InstDyn>(W, L.instd);
    d.glob = at<Globals>(W, L.glob);
    d.seg_tile0 = at<int64_t>(W, L.seg_tile0);
    d.seg_base = at<int64_t>(W, L.seg_base);
    d.inst_ftile0 = at<int64_t>(W, L.inst_ftile0);
    d.node_base = at<int64_t>(W, L.node_base);
    d.S = at<unsigned long long>(W, L.S);
    d.rho = at<double>(W, L.rho);
    d.phi = at<double>(W, L.phi);
    d.E = at<double>(W, L.E);
    d.dprime = at<double>(W, L.dprime);
    d.acc64 = at<double>(W, L.acc64);
    d.acc32 = at<float>(W, L.acc32);
    d.hist = at<uint32_t>(W, L.hist);
    d.cursor = at<uint32_t>(W, L.cursor);
    d.offsets = at<uint32_t>(W, L.offsets);
    d.seg_start = at<unsigned long long>(W, L.seg_start);
    d.fwd_status = at<AffineStatus>(W, L.fwd_status);
    d.bwd_status = at<BackStatus>(W, L.bwd_status);
    d.sweep = at<NodeSweep>(W, L.sweep);
    d.bpre = at<BackStatus>(W, L.bpre);
    d.sort_status = at<unsigned long long>(W, L.sort_status);
    d.fe_part = at<double>(W, L.fe_part);
    d.cand = at<Cand>(W, L.cand);
    d.cand_n = at<uint32_t>(W, L.cand_n);
    d.ev = at<IzEvent>(W, L.ev);
    d.ev_n = at<uint32_t>(W, L.ev_n);
    d.ev_rank = at<uint32_t>(W, L.ev_rank);
    d.ev_crank = at<uint32_t>(W, L.ev_crank);
    d.ev_target = at<long long>(W, L.ev_target);
    d.nn = at<double>(W, L.nn);
    d.ev_pre = at<uint32_t>(W, L.ev_pre);
    d.inst_ev = at<uint32_t>(W, L.inst_ev);
    d.inst_fill = at<uint32_t>(W, L.inst_fill);
    d.inst_start = at<uint32_t>(W, L.inst_start);
    d.rank_bucket = at<RankEntry>(W, L.rank_bucket);
    d.cnt_slot = at<unsigned long long>(W, L.cnt_slot);
    d.diag_part = at<double>(W, L.diag_part);
    d.diag_out = at<pic_diag>(W, L.diag_out);
    d.n_slots = p.n_slots;
    d.n_tiles = p.n_tiles;
    d.G = p.G;
    d.cand_ovf_cap = L.cand_ovf_cap;
    d.ev_ovf_cap = L.ev_ovf_cap;
    d.cand_q = (int32_t)L.cand_q;
    d.ev_q = (int32_t)L.ev_q;
    d.n_push_blocks = p.n_push_blocks;
    d.n_regions = p.n_regions;
    c->default_blocks = p.n_push_blocks;
    d.n_field_tiles = p.n_field_tiles;
    d.n_sort_tiles = p.n_sort_tiles;
    d.n_seg = n_seg;
    d.n_inst = n_inst;
    d.nsp = nsp;
    d.precision = c->precision;
    // The FP32 mover's deposit window: with a deposit array that fits in one
    // XCD's 4 MiB L2 its flush is issued after the next pass's loads, where
    // its atomics no longer hold those loads up; with a larger one the
    // atomics take longer, and issued there they hold up the gathers' wait
    // instead, so the flush stays at the end of the pass.  (Bench workload,
    // 1.6 MB: step 0.2650 -> 0.2620 ms; 10^6 cells, 16 MB: 4.95 -> 5.10 ms.)
    d.late_flush = (uint64_t)nsp * (uint64_t)p.G * sizeof(unsigned long long) <= (4ull << 20) ? 1 : 0;
    d.kinetic_any = 0;
    d.field_all_off = 1;
    for (int i = 0; i < n_inst; ++i) {
        if (find_kind(cfgs[i], PIC_KIND_NEUTRAL) >= 0) d.kinetic_any = 1;
        if (!cfgs[i].field_off) d.field_all_off = 0;
    }

    hipStream_t st = c->st;
    bool ok = hipMemsetAsync(W, 0, L.total, st) == hipSuccess;
    ok = ok && hipMemcpyAsync((void *)d.segc, segc.data(), sizeof(SegConst) * n_seg,
                              hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync((void *)d.instc, instc.data(), sizeof(InstConst) * n_inst,
                              hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(d.segd, segd.data(), sizeof(SegDyn) * n_seg, hipMemcpyHostToDevice,
                              st) == hipSuccess;
    ok = ok && hipMemcpyAsync(d.instd, instd.data(), sizeof(InstDyn) * n_inst,
                              hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(d.glob, &g, sizeof(Globals), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync((void *)d.seg_tile0, p.seg_tile0.data(), sizeof(int64_t) * (n_seg + 1),
                              hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync((void *)d.seg_base, p.seg_base.data(), sizeof(int64_t) * (n_seg + 1),
                              hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync((void *)d.inst_ftile0, p.inst_ftile0.data(),
                              sizeof(int64_t) * (n_inst + 1), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync((void *)d.node_base, p.node_base.data(), sizeof(int64_t) * (n_inst + 1),
                              hipMemcpyHostToDevice, st) == hipSuccess;
    // the host vectors above must stay alive until the copies are done
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (ok && (flags & PIC_INIT_DEVICE)) ok = launch_init_device(d, st) == hipSuccess;
    ok = ok && launch_init_state(d, st, nullptr) == hipSuccess;
    if (ok && (flags & PIC_INIT_SORT)) ok = launch_sort(d, st) == hipSuccess;
    if (ok && !(flags & PIC_INIT_NO_FIELD)) {
        ok = launch_deposit(d, st) == hipSuccess;
        ok = ok && launch_field(d, st, c->max_smooth) == hipSuccess;
    }
    if (pinned_diag) {
        ok = ok && hipHostMalloc((void **)&c->host_diag, sizeof(pic_diag) * n_inst,
                                 hipHostMallocDefault) == hipSuccess;
        c->host_diag_pinned = true;
    } else {
        c->diag_stage.resize(n_inst);
        c->host_diag = c->diag_stage.data();
    }
    if (!ok) {
        if (c->host_diag && c->host_diag_pinned) (void)hipHostFree(c->host_diag);
        delete c;
        return PIC_E_DEVICE;
    }
    *out = c;
    return PIC_OK;
}

void mark_static(pic_ctx *c, int device) { c->static_dev = device; }

}  // namespace picx

extern "C" {

int pic_init(const pic_config *cfgs, int n_inst, const pic_buffers *bufs, void *stream,
             unsigned flags, pic_ctx **out)
{
    if (!bufs) {
        if (out) *out = nullptr;
        return PIC_E_ARG;
    }
    return init_context(cfgs, n_inst, bufs, bufs->work, stream, flags, true, out);
}

int pic_push(pic_ctx *c, unsigned flags)
{
    if (!c) return PIC_E_STATE;
    const bool dep = !(flags & PIC_PUSH_NO_DEPOSIT);
    return launch_push(c->d, c->st, dep, c->mcc_any, c->sub_any, c->chunks, false) == hipSuccess
               ? PIC_OK
               : PIC_E_DEVICE;
}

int pic_deposit(pic_ctx *c)
{
    if (!c) return PIC_E_STATE;
    return launch_deposit(c->d, c->st) == hipSuccess ? PIC_OK : PIC_E_DEVICE;
}

int pic_field_solve(pic_ctx *c)
{
    if (!c) return PIC_E_STATE;
    return launch_field(c->d, c->st, c->max_smooth) == hipSuccess ? PIC_OK : PIC_E_DEVICE;
}

int pic_mcc_collide(pic_ctx *c)
{
    if (!c) return PIC_E_STATE;
    if (c->mcc_any && launch_collide(c->d, c->st, false) != hipSuccess) return PIC_E_DEVICE;
    if (launch_emit(c->d, c->st, c->mcc_any || c->src_any, c->mcc_any) != hipSuccess) return PIC_E_DEVICE;
    c->host_steps += 1;
    return PIC_OK;
}

int pic_sort(pic_ctx *c)
{
    if (!c) return PIC_E_STATE;
    return launch_sort(c->d, c->st) == hipSuccess ? PIC_OK : PIC_E_DEVICE;
}

}  // extern "C"

namespace {

// pic_push, pic_mcc_collide and pic_field_solve, with the same results: with
// collisions on, each mover block collides its own region's candidates right
// after its push, and the collide kernel takes only the shared overflow list;
// with no periodic instance the close of the step runs as one more block of
// the field's first launch instead of a launch of its own
int step_once(pic_ctx *c)
{
    int close_mode = -1;
    int *defer = c->periodic_any ? nullptr : &close_mode;
    bool ok;
    if (!c->mcc_any) {
        const int rc = pic_push(c, 0);
        if (rc) return rc;
        ok = launch_emit(c->d, c->st, c->src_any, false, defer) == hipSuccess;
    } else {
        ok = launch_push(c->d, c->st, true, true, c->sub_any, c->chunks, true) == hipSuccess &&
             launch_collide(c->d, c->st, true) == hipSuccess &&
             launch_emit(c->d, c->st, true, true, defer) == hipSuccess;
    }
    ok = ok && launch_field(c->d, c->st, c->max_smooth, close_mode) == hipSuccess;
    if (!ok) return PIC_E_DEVICE;
    c->host_steps += 1;
    return PIC_OK;
}

}  // namespace

extern "C" {

int pic_step(pic_ctx *c, int n_steps, int sort_every)
{
    if (!c) return PIC_E_STATE;
    if (n_steps < 0 || sort_every < 0) return PIC_E_ARG;
    for (int s = 0; s < n_steps; ++s) {
        int rc = step_once(c);
        if (!rc && sort_every > 0 && ((c->cfg[0].step0 + c->host_steps) % sort_every) == 0)
            rc = pic_sort(c);
        if (rc) return rc;
    }
    return PIC_OK;
}

namespace {

// enqueue `n` whole steps on c->st, the sort after the last one when `sort`
int enqueue_period(pic_ctx *c, int n, bool sort)
{
    for (int s = 0; s < n; ++s) {
        const int rc = step_once(c);
        if (rc) return rc;
    }
    return sort ? pic_sort(c) : PIC_OK;
}

void drop_graph(pic_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->g_period = 0;
    c->g_sort = -1;
    c->g_phase = 0;
}

// steps since the last multiple of the cadence (0 without sorting)
int cadence_phase(const pic_ctx *c, int sort_every)
{
    return sort_every > 0 ? (int)((c->cfg[0].step0 + c->host_steps) % sort_every) : 0;
}

// capture one period (sort_every steps and the sort, or one step when
// sort_every is 0) into c->gexec, starting at `phase` steps into the
// cadence: sort_every - phase steps, the sort, then the other phase steps
int capture_period(pic_ctx *c, int sort_every, int phase)
{
    drop_graph(c);
    if (!c->cap_st && hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking) != hipSuccess) {
        c->cap_st = nullptr;
        return PIC_E_DEVICE;
    }
    const int period = sort_every > 0 ? sort_every : 1;
    hipStream_t user = c->st;
    const int64_t steps = c->host_steps;
    if (hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return PIC_E_DEVICE;
    c->st = c->cap_st;
    int rc = enqueue_period(c, period - phase, sort_every > 0);
    if (!rc && phase > 0) rc = enqueue_period(c, phase, false);
    c->st = user;
    c->host_steps = steps;  // capture enqueues nothing
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_st, &g);
    if (rc || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : PIC_E_DEVICE;
    }
    const hipError_t ei = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        c->gexec = nullptr;
        return PIC_E_DEVICE;
    }
    c->g_period = period;
    c->g_sort = sort_every;
    c->g_phase = phase;
    return PIC_OK;
}

}  // namespace

int pic_step_graph(pic_ctx *c, int n_steps, int sort_every)
{
    if (!c) return PIC_E_STATE;
    if (n_steps < 0 || sort_every < 0) return PIC_E_ARG;
    int left = n_steps;
    // whole periods from the current phase of the cadence replay one graph
    // (its sort where pic_step would sort); the remainder runs eagerly.
    // n_steps = 0: capture and upload that graph only, launching nothing
    const int period = sort_every > 0 ? sort_every : 1;
    const int phase = cadence_phase(c, sort_every);
    if ((left >= period || n_steps == 0) &&
        (!c->gexec || c->g_sort != sort_every || c->g_phase != phase)) {
        const int rc = capture_period(c, sort_every, phase);
        if (rc) return rc;
        if (n_steps == 0 && hipGraphUpload(c->gexec, c->st) != hipSuccess) return PIC_E_DEVICE;
    }
    while (left >= period) {
        if (hipGraphLaunch(c->gexec, c->st) != hipSuccess) return PIC_E_DEVICE;
        c->host_steps += period;
        left -= period;
    }
    return left > 0 ? pic_step(c, left, sort_every) : PIC_OK;
}

int pic_set_mover(pic_ctx *c, int chunks, int blocks)
{
    if (!c) return PIC_E_STATE;
    if (chunks != kPer && chunks != kPer / 2) return PIC_E_ARG;
    if (blocks == 0) blocks = c->default_blocks;
    if (blocks < 1 || blocks > c->d.n_regions) return PIC_E_ARG;
    if (chunks != c->chunks || blocks != c->d.n_push_blocks) drop_graph(c);
    c->chunks = chunks;
    c->d.n_push_blocks = blocks;
    return PIC_OK;
}

namespace {

// sort, then trial_steps whole steps at `cadence` as in pic_step_graph, timed
// with HIP events on the context's stream: particle-steps per second
int time_trial(pic_ctx *c, int trial_steps, int cadence, hipEvent_t e0, hipEvent_t e1, double *rate)
{
    std::vector<InstDyn> before(c->n_inst), after(c->n_inst);
    int rc = pic_sort(c);  // every trial starts from freshly sorted particles
    if (rc) return rc;
    // the graph of this cadence is captured and uploaded before the timing
    const int phase = cadence_phase(c, cadence);
    if (trial_steps >= (cadence > 0 ? cadence : 1) &&
        (!c->gexec || c->g_sort != cadence || c->g_phase != phase)) {
        rc = capture_period(c, cadence, phase);
        if (rc) return rc;
        if (hipGraphUpload(c->gexec, c->st) != hipSuccess) return PIC_E_DEVICE;
    }
    if (hipMemcpyAsync(before.data(), c->d.instd, sizeof(InstDyn) * c->n_inst, hipMemcpyDeviceToHost,
                       c->st) != hipSuccess ||
        hipEventRecord(e0, c->st) != hipSuccess)
        return PIC_E_DEVICE;
    rc = pic_step_graph(c, trial_steps, cadence);
    if (rc) return rc;
    if (hipEventRecord(e1, c->st) != hipSuccess ||
        hipMemcpyAsync(after.data(), c->d.instd, sizeof(InstDyn) * c->n_inst, hipMemcpyDeviceToHost,
                       c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
        return PIC_E_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f)) return PIC_E_DEVICE;
    double ps = 0.0;
    for (int k = 0; k < c->n_inst; ++k)
        ps += (double)(after[k].particle_steps - before[k].particle_steps);
    *rate = ps / (1e-3 * (double)ms);
    return PIC_OK;
}

struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = false;
    EventPair()
    {
        ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    }
    ~EventPair()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Each of n configurations (set(i, &cadence) selects configuration i and
// its sort cadence) is timed in kTuneRounds interleaved rounds after one
// untimed warm-up trial of the first; rate[i] = its best round.  (The first
// trials after a quiet spell ran slower than later ones, which favoured the
// configurations timed last.)
constexpr int kTuneRounds = 2;

}  // namespace
}  // extern "C"

namespace {

template <class Set>
int best_of_rounds(pic_ctx *c, int n, int trial_steps, EventPair &ev, double *rate, Set set)
{
    int cadence = 0;
    int rc = set(0, &cadence);
    double r = 0.0;
    if (!rc) rc = time_trial(c, trial_steps, cadence, ev.e0, ev.e1, &r);
    for (int round = 0; round < kTuneRounds && !rc; ++round)
        for (int i = 0; i < n && !rc; ++i) {
            rc = set(i, &cadence);
            if (!rc) rc = time_trial(c, trial_steps, cadence, ev.e0, ev.e1, &r);
            if (!rc && r > rate[i]) rate[i] = r;
        }
    return rc;
}

}  // namespace

extern "C" {

int pic_autotune_sort(pic_ctx *c, const int *cand, int n_cand, int trial_steps, int *best,
                      double *rates)
{
    if (!c) return PIC_E_STATE;
    if (!cand || n_cand < 1 || trial_steps < 1 || !best) return PIC_E_ARG;
    for (int i = 0; i < n_cand; ++i)
        if (cand[i] < 0) return PIC_E_ARG;
    EventPair ev;
    if (!ev.ok) return PIC_E_DEVICE;
    std::vector<double> r(n_cand, -1.0);
    const int rc = best_of_rounds(c, n_cand, trial_steps, ev, r.data(),
                                  [&](int i, int *cadence) { *cadence = cand[i]; return PIC_OK; });
    if (rc) return rc;
    int pick = 0;
    for (int i = 0; i < n_cand; ++i) {
        if (rates) rates[i] = r[i];
        if (r[i] > r[pick]) pick = i;
    }
    *best = cand[pick];
    return PIC_OK;
}

int pic_autotune(pic_ctx *c, const int *chunks, const int *blocks, int n_movers, const int *cadences,
                 int n_cad, int trial_steps, int *best_mover, int *best_cadence, double *rates)
{
    if (!c) return PIC_E_STATE;
    if (!chunks || !blocks || n_movers < 1 || !cadences || n_cad < 1 || trial_steps < 1 ||
        !best_mover || !best_cadence)
        return PIC_E_ARG;
    for (int i = 0; i < n_movers; ++i) {
        const int b = blocks[i] == 0 ? c->default_blocks : blocks[i];
        if ((chunks[i] != kPer && chunks[i] != kPer / 2) || b < 1 || b > c->d.n_regions)
            return PIC_E_ARG;
    }
    for (int i = 0; i < n_cad; ++i)
        if (cadences[i] < 0) return PIC_E_ARG;
    EventPair ev;
    if (!ev.ok) return PIC_E_DEVICE;
    // the mover configurations at the first cadence
    std::vector<double> rm(n_movers, -1.0);
    int rc = best_of_rounds(c, n_movers, trial_steps, ev, rm.data(), [&](int i, int *cadence) {
        *cadence = cadences[0];
        return pic_set_mover(c, chunks[i], blocks[i]);
    });
    if (rc) return rc;
    int pick = 0;
    for (int i = 0; i < n_movers; ++i) {
        if (rates) rates[i] = rm[i];
        if (rm[i] > rm[pick]) pick = i;
    }
    *best_mover = pick;
    rc = pic_set_mover(c, chunks[pick], blocks[pick]);
    if (rc) return rc;
    // then the cadences with that mover
    std::vector<double> rcad(n_cad, -1.0);
    rc = best_of_rounds(c, n_cad, trial_steps, ev, rcad.data(),
                        [&](int j, int *cadence) { *cadence = cadences[j]; return PIC_OK; });
    if (rc) return rc;
    int cpick = 0;
    for (int j = 0; j < n_cad; ++j) {
        if (rates) rates[n_movers + j] = rcad[j];
        if (rcad[j] > rcad[cpick]) cpick = j;
    }
    *best_cadence = cadences[cpick];
    return PIC_OK;
}

int pic_diagnostics(pic_ctx *c, pic_diag *out, int n_inst)
{
    if (!c) return PIC_E_STATE;
    if (!out || n_inst != c->n_inst) return PIC_E_ARG;
    if (launch_diag(c->d, c->st) != hipSuccess) return PIC_E_DEVICE;
    if (hipMemcpyAsync(c->host_diag, c->d.diag_out, sizeof(pic_diag) * n_inst,
                       hipMemcpyDeviceToHost, c->st) != hipSuccess)
        return PIC_E_DEVICE;
    if (hipStreamSynchronize(c->st) != hipSuccess) return PIC_E_DEVICE;
    std::memcpy(out, c->host_diag, sizeof(pic_diag) * n_inst);
    uint32_t st = 0;
    for (int i = 0; i < n_inst; ++i) st |= out[i].status;
    return status_code(st);
}

int pic_region(const pic_ctx *c, int region, uint64_t *byte_offset, int64_t *n_elems)
{
    if (!c || !byte_offset || !n_elems) return PIC_E_ARG;
    const Layout &L = c->L;
    const int64_t G = c->d.G, nb = (int64_t)c->nsp * G;
    switch (region) {
    case PIC_R_DEPOSIT: *byte_offset = L.S; *n_elems = nb; break;
    case PIC_R_RHO: *byte_offset = L.rho; *n_elems = G; break;
    case PIC_R_PHI: *byte_offset = L.phi; *n_elems = G; break;
    case PIC_R_EFIELD: *byte_offset = L.E; *n_elems = G; break;
    case PIC_R_ACC64: *byte_offset = L.acc64; *n_elems = nb; break;
    case PIC_R_ACC32: *byte_offset = L.acc32; *n_elems = nb; break;
    case PIC_R_CELL_OFFSETS: *byte_offset = L.offsets; *n_elems = nb; break;
    case PIC_R_NODE_BASE: *byte_offset = L.node_base; *n_elems = c->n_inst + 1; break;
    case PIC_R_NEUTRAL_DENSITY: *byte_offset = L.nn; *n_elems = G; break;
    default: return PIC_E_ARG;
    }
    return PIC_OK;
}

int pic_destroy(pic_ctx *c)
{
    if (!c) return PIC_E_ARG;
    drop_graph(c);
    if (c->cap_st) (void)hipStreamDestroy(c->cap_st);
    if (c->host_diag && c->host_diag_pinned) (void)hipHostFree(c->host_diag);
    if (c->static_dev >= 0) static_release(c->static_dev);
    delete c;
    return PIC_OK;
}

const char *pic_strerror(int code)
{
    switch (code) {
    case PIC_OK: return "ok";
    case PIC_E_ARG: return "invalid argument";
    case PIC_E_CONFIG: return "invalid configuration";
    case PIC_E_DEVICE: return "HIP runtime error";
    case PIC_E_CAPACITY: return "particle capacity exceeded";
    case PIC_E_CFL: return "|vx| reached one cell per step";
    case PIC_E_NONFINITE: return "non-finite particle velocity";
    case PIC_E_STATE: return "call out of order or inconsistent device state";
    case PIC_E_SCRATCH:
        return "workspace larger than the library's static scratch array (PIC_STATIC_WORK_MAX)";
    case PIC_E_BUSY: return "the device's static scratch array is held by another context";
    default: return "unknown error";
    }
}

}  // extern "C"
