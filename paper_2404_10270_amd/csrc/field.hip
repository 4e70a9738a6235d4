// field.hip -- the field solver (paper Sec. 2, phase 3) in FP64 on gfx950.
//
//   rho_j = sum_s q_s w_s S_s[j] 2^-32 / V_j   (+ a uniform background when periodic)
//   phi_{j-1} - 2 phi_j + phi_{j+1} = -rho_j dx^2 / eps0,  j = 1..nc-1,  phi_0 = phi_nc = 0
//   E_j = (phi_{j-1} - phi_{j+1}) / (2 dx), wall nodes closed by Gauss's law over
//   their half cell (absorbing walls) or wrapped (periodic), acc_s = (q_s/m_s) E dt^2/dx.
//
// The tridiagonal system is solved with the Thomas algorithm.  Its two sweeps
// are first-order linear recurrences,
//   forward   d'_u = (u/(u+1)) d'_{u-1} - (u/(u+1)) d_u     (pivots of [1,-2,1]:
//                                                             c'_u = g_u = -u/(u+1))
//   backward  phi_u = (u/(u+1)) phi_{u+1} + d'_u,
// so each sweep is evaluated as a scan over affine maps y -> A y + B: every
// thread composes kFieldR consecutive maps and the block scans the thread
// maps.  A tile's backward composite depends on the d' entering it from
// below only linearly (d' = d'(0) + h y, with d'(0) the sweep entering with
// 0 and h the sweep of 1 with no sources), so both sweeps need a single
// exchange between tiles and the solve takes two launches, with no atomics
// and no waiting between blocks:
//   1. rho; each tile's forward composite and its backward composite as a
//      function of the d' entering it; each node's d'(0) and h, and each
//      thread's composite of the backward maps above its nodes in the tile;
//   2. every block scans the tiles' composites of its instance: the d'
//      entering its tile from below and the phi entering it from above; then
//      each thread's d' = d'(0) + h y and phi with no scan inside the tile,
//      E, the accelerations and the field energy.
// Same recurrences as the sequential sweep, regrouped; only the rounding
// order differs.
//
// The first launch also forms the node density of a kinetic neutral species,
//   n_j = w_n S_n[j] 2^-32 / V_j,
// which the collisions gather at the electrons.  An instance without a field
// solve (the paper's Table 1 case) gets E = phi = 0; when no instance solves
// the field, the first launch alone runs (rho, the neutral density, the
// deposit cleared).  Inside a whole step with no periodic instance, the
// first launch takes one block more, which closes the step (step_close.h):
// nothing else in the solve reads what the close writes.
#include "device_common.h"
#include "step_close.h"

#pragma clang fp contract(off)

namespace picx {

struct Aff {
    double A, B;
};

// apply `first`, then `second`
__device__ __forceinline__ Aff compose(Aff second, Aff first)
{
    Aff r;
    r.A = second.A * first.A;
    r.B = second.A * first.B + second.B;
    return r;
}

// a backward map whose constant is B0 + B1 y for the d' y entering the tile
struct Aff3 {
    double A, B0, B1;
};

__device__ __forceinline__ Aff3 compose3(Aff3 second, Aff3 first)
{
    Aff3 r;
    r.A = second.A * first.A;
    r.B0 = second.A * first.B0 + second.B0;
    r.B1 = second.A * first.B1 + second.B1;
    return r;
}

__device__ __forceinline__ Aff shfl_up_aff(Aff a, int d)
{
    Aff r;
    r.A = __shfl_up(a.A, d, 64);
    r.B = __shfl_up(a.B, d, 64);
    return r;
}

// exclusive scan of thread maps in thread order over the block; returns the
// composition of all maps of lower threads (identity for thread 0) and writes
// the block aggregate to *agg (all threads)
__device__ Aff block_exclusive_scan(Aff m, Aff *agg)
{
    __shared__ Aff s_wave[kWaves];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    Aff inc = m;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const Aff o = shfl_up_aff(inc, d);
        if (lane >= d) inc = compose(inc, o);
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    Aff wpre = {1.0, 0.0};
    for (int w = 0; w < wave; ++w) wpre = compose(s_wave[w], wpre);
    Aff total = {1.0, 0.0};
    for (int w = 0; w < kWaves; ++w) total = compose(s_wave[w], total);
    Aff excl = shfl_up_aff(inc, 1);
    if (lane == 0) excl = Aff{1.0, 0.0};
    *agg = total;
    __syncthreads();
    return compose(excl, wpre);
}

// -g_u = u/(u+1): the multiplier of both sweeps at node u
__device__ __forceinline__ double gq_of(int64_t j)
{
    const double u = (double)j;
    return u / (u + 1.0);
}

// ---------------------------------------------------------------------------
// 1. rho and the forward composite of every tile
// ---------------------------------------------------------------------------
enum { kRhoSolve = 0, kRhoFromRho = 1, kRhoNoSolve = 2 };

// mode kRhoSolve: rho (and the neutral density) from the deposit, and the
// composites; kRhoFromRho: rho is already in place (smoothed), only the
// composites; kRhoNoSolve: rho and the neutral density, the deposit cleared,
// no composites (no instance solves the field).  CLOSE: the last block
// closes the step instead (close_step, mode close_mode).
template <bool CLOSE>
__global__ __launch_bounds__(kBlock) void field_rho_kernel(Dev d, int mode, int close_mode)
{
    if constexpr (CLOSE) {
        if (blockIdx.x == gridDim.x - 1) {  // block-uniform
            close_step(d, close_mode);
            return;
        }
    }
    const bool from_rho = (mode == kRhoFromRho);
    const int64_t vt = blockIdx.x;
    const int inst = seg_of_tile(d.inst_ftile0, d.n_inst, vt);
    const InstConst &ic = d.instc[inst];
    const int64_t lt = vt - ic.ftile0;
    const int nc = ic.nc;
    const bool periodic = (ic.bc == PIC_BC_PERIODIC);
    const int64_t G = d.G;
    const int nsp = ic.nsp;
    const double two_m32 = 0x1p-32;
    // the instance's constants read once (the stores to rho below would make
    // the compiler read them again, with a wait, per node)
    const int64_t gnode = ic.gnode;
    const double dx = ic.dx, K = ic.K;

    // uniform background for periodic systems, from the live counts
    double rho_bg = 0.0;
    if (periodic) {
        double qn = 0.0;
        for (int k = 0; k < nsp; ++k) qn += d.segc[ic.seg0 + k].qw * (double)d.segd[ic.seg0 + k].live;
        rho_bg = -qn / ((double)nc * dx);
    }

    const int64_t j0 = lt * kFieldTile + (int64_t)threadIdx.x * kFieldR;
    // the deposit of the thread's nodes for every species, and of nodes 0 and
    // nc (the periodic wrap), loaded before the first wait: unpredicated, a
    // node past nc reads node nc and a species past nsp repeats the last one,
    // neither used
    unsigned long long Sv[kFieldR][PIC_MAX_SPECIES], S0[PIC_MAX_SPECIES], Snc[PIC_MAX_SPECIES];
    double qw[PIC_MAX_SPECIES];  // q w of each species (read once, not per node)
    if (!from_rho) {
#pragma unroll
        for (int k = 0; k < PIC_MAX_SPECIES; ++k) {
            const int kk = min(k, nsp - 1);
            const unsigned long long *Sk = d.S + kk * G + gnode;
#pragma unroll
            for (int r = 0; r < kFieldR; ++r) Sv[r][k] = Sk[min(j0 + r, (int64_t)nc)];
            S0[k] = Sk[0];
            Snc[k] = Sk[nc];
            qw[k] = d.segc[ic.seg0 + kk].qw;
        }
    }
    const double wn = ic.seg_n >= 0 ? d.segc[ic.seg_n].w : 0.0;  // the atoms' weight
    const int spn = ic.seg_n >= 0 ? d.segc[ic.seg_n].sp : -1;
    // the deposit at node j of species k, with the periodic wrap
    auto dep_at = [&](int r, int k, int64_t j) -> unsigned long long {
        unsigned long long Sj = Sv[r][k];
        if (periodic) {
            if (j == 0) Sj += Snc[k];
            if (j == nc) Sj = S0[k] + Snc[k];
        }
        return Sj;
    };
    Aff m = {1.0, 0.0};
    double dv[kFieldR];  // d_j = -rho_j K of the thread's interior nodes
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) {
        const int64_t j = j0 + r;
        dv[r] = 0.0;
        if (j > nc) continue;
        if (from_rho) {
            if (j >= 1 && j <= nc - 1) {
                const double dd = -(d.rho[gnode + j] * K);
                dv[r] = dd;
                const double gq = gq_of(j);
                m = compose(Aff{gq, -(gq * dd)}, m);
            }
            continue;
        }
        // without a solve the deposit is cleared in this launch: on a periodic
        // grid node 0's thread also writes node nc (the same node) and no
        // thread reads node nc's deposit after it is cleared
        if (mode == kRhoNoSolve && periodic && j == nc) continue;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < PIC_MAX_SPECIES; ++k)
            if (k < nsp) acc += qw[k] * ((double)dep_at(r, k, j) * two_m32);
        double V = dx;
        if (!periodic && (j == 0 || j == nc)) V = 0.5 * dx;
        const double rho = acc / V + rho_bg;
        d.rho[gnode + j] = rho;
        if (mode == kRhoNoSolve && periodic && j == 0) d.rho[gnode + nc] = rho;
        if (d.kinetic_any) {
            double n = 0.0;
            if (ic.seg_n >= 0) {
                unsigned long long Sj = 0;
#pragma unroll
                for (int k = 0; k < PIC_MAX_SPECIES; ++k)
                    if (k == spn) Sj = dep_at(r, k, j);
                n = (wn * ((double)Sj * two_m32)) / V;
            }
            d.nn[gnode + j] = n;
            if (mode == kRhoNoSolve && periodic && j == 0) d.nn[gnode + nc] = n;
        }
        if (mode == kRhoNoSolve) continue;
        if (j >= 1 && j <= nc - 1) {
            const double dd = -(rho * K);
            dv[r] = dd;
            const double gq = gq_of(j);
            m = compose(Aff{gq, -(gq * dd)}, m);
        }
    }
    if (mode == kRhoNoSolve) {
        // the deposit is consumed; E, phi and the accelerations stay zero
        // (cleared at set-up, never written in this mode)
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kFieldR; ++r) {
            const int64_t j = j0 + r;
            if (j > nc || (periodic && j == nc)) continue;
            for (int k = 0; k < nsp; ++k) {
                d.S[k * G + gnode + j] = 0ull;
                if (periodic && j == 0) d.S[k * G + gnode + nc] = 0ull;
            }
        }
        if (threadIdx.x == 0) d.fe_part[vt] = 0.0;
        return;
    }
    Aff agg;
    const Aff excl = block_exclusive_scan(m, &agg);
    if (threadIdx.x == 0) {
        d.fwd_status[vt].A = agg.A;
        d.fwd_status[vt].B = agg.B;
    }
    // the forward sweep inside the tile entering with 0 (d0: the tile's own
    // sources) and entering with 1 without sources (h): d' = d0 + h y
    double d0[kFieldR], h[kFieldR];
    double y0 = excl.B, y1 = excl.A;
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) {
        const int64_t j = j0 + r;
        d0[r] = h[r] = 0.0;
        if (j >= 1 && j <= nc - 1) {
            const double gq = gq_of(j);
            y0 = gq * y0 + (-(gq * dv[r]));
            y1 = gq * y1;
            d0[r] = y0;
            h[r] = y1;
        }
    }
    // backward maps phi_u = (u/(u+1)) phi_{u+1} + d'_u of the thread's nodes,
    // top first, with the constant split as d'
    Aff3 mb = {1.0, 0.0, 0.0};
#pragma unroll
    for (int r = kFieldR - 1; r >= 0; --r) {
        const int64_t j = j0 + r;
        if (j >= 1 && j <= nc - 1) mb = compose3(Aff3{gq_of(j), d0[r], h[r]}, mb);
    }
    // the nodes' forward terms, for the second launch
    NodeSweep *sw = d.sweep + vt * kFieldTile + (int64_t)threadIdx.x * kFieldR;
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) sw[r] = NodeSweep{d0[r], h[r]};
    // the backward maps of the threads above each thread (a scan from the top
    // of the tile down), and the tile's composite: inside a wave, lane l
    // takes the lanes above it, s at a time
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    Aff3 inc = mb;  // this lane's map after those of the lanes above it
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        Aff3 o;
        o.A = __shfl_down(inc.A, s, 64);
        o.B0 = __shfl_down(inc.B0, s, 64);
        o.B1 = __shfl_down(inc.B1, s, 64);
        if (lane + s < 64) inc = compose3(inc, o);
    }
    Aff3 ex;  // the lanes above this one
    ex.A = __shfl_down(inc.A, 1, 64);
    ex.B0 = __shfl_down(inc.B0, 1, 64);
    ex.B1 = __shfl_down(inc.B1, 1, 64);
    if (lane == 63) ex = Aff3{1.0, 0.0, 0.0};
    __shared__ Aff3 s_b[kWaves];
    if (lane == 0) s_b[wave] = inc;  // the wave's composite
    __syncthreads();
    Aff3 above = {1.0, 0.0, 0.0};  // the waves above this one, top first
    for (int w = kWaves - 1; w > wave; --w) above = compose3(s_b[w], above);
    const Aff3 pre = compose3(ex, above);
    d.bpre[vt * kBlock + threadIdx.x] = BackStatus{pre.A, pre.B0, pre.B1};
    if (threadIdx.x == 0) {
        const Aff3 r = compose3(inc, above);
        d.bwd_status[vt].A = r.A;
        d.bwd_status[vt].B0 = r.B0;
        d.bwd_status[vt].B1 = r.B1;
    }
}

// The values entering tile lt of an instance (ntl tiles from tile `first`):
// y_in, the d' entering it from below; phi_above, the phi entering it from
// above (the backward composites of the tiles above, top first, applied to
// phi_nc = 0, each with the d' entering that tile); dp_top, the d' leaving
// the last tile (at node nc - 1).  Every thread takes a run of consecutive
// tiles: a block scan of the runs' forward composites gives the d' entering
// each run, a second one, over the runs from the top, the backward
// composites above each run.  Runs of up to kRunR tiles (instances of up to
// kRunR x kBlock tiles) are read into registers before the first wait.  All
// threads; barriers inside.
constexpr int kRunR = 4;

template <int R>
__device__ void tile_level_r(const Dev &d, int64_t first, int64_t ntl, int64_t lt, double &y_in,
                             double &phi_above, double &dp_top)
{
    __shared__ double s_y[kBlock];  // d' entering each run
    __shared__ double s_out[2];
    const int64_t per = (ntl + kBlock - 1) / kBlock;
    const int64_t n_runs = (ntl + per - 1) / per;
    // thread t: forward run t, backward run n_runs - 1 - t (runs of `per` tiles)
    const int64_t a0 = (int64_t)threadIdx.x * per;
    const int64_t a1 = min(a0 + per, ntl);
    const int64_t q = n_runs - 1 - (int64_t)threadIdx.x;
    const int64_t b0 = q >= 0 ? q * per : 0;
    const int64_t b1 = q >= 0 ? min(b0 + per, ntl) : 0;
    const AffineStatus one = {1.0, 0.0};
    const BackStatus bone = {1.0, 0.0, 0.0};
    AffineStatus F[R], FB[R];
    BackStatus B[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        F[i] = (a0 + i < a1) ? d.fwd_status[first + a0 + i] : one;
        FB[i] = (b0 + i < b1) ? d.fwd_status[first + b0 + i] : one;
        B[i] = (b0 + i < b1) ? d.bwd_status[first + b0 + i] : bone;
    }
    // forward
    Aff m = {1.0, 0.0};
#pragma unroll
    for (int i = 0; i < R; ++i)
        if (a0 + i < a1) m = compose(Aff{F[i].A, F[i].B}, m);
    Aff agg;
    const Aff ex = block_exclusive_scan(m, &agg);
    s_y[threadIdx.x] = ex.B;  // applied to d'_0 = 0
    if (a0 <= lt && lt < a1) {
        double y = ex.B;
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (a0 + i < lt) y = F[i].A * y + F[i].B;
        s_out[0] = y;
    }
    __syncthreads();
    // backward: each tile's map with the d' entering it, from the top down
    Aff bk[R];
    {
        double y = q >= 0 ? s_y[q] : 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            bk[i] = Aff{B[i].A, B[i].B0 + B[i].B1 * y};
            y = FB[i].A * y + FB[i].B;
        }
    }
    Aff mb = {1.0, 0.0};
#pragma unroll
    for (int i = R - 1; i >= 0; --i)
        if (b0 + i < b1) mb = compose(bk[i], mb);
    Aff aggb;
    const Aff exb = block_exclusive_scan(mb, &aggb);
    if (q >= 0 && b0 <= lt && lt < b1) {
        Aff M = exb;
#pragma unroll
        for (int i = R - 1; i >= 0; --i)
            if (b0 + i < b1 && b0 + i > lt) M = compose(bk[i], M);
        s_out[1] = M.B;
    }
    __syncthreads();
    y_in = s_out[0];
    phi_above = s_out[1];
    dp_top = agg.B;
}

// the same inside every wave on its own (no LDS, no barrier), for instances
// of up to 64 R tiles: lane l takes runs of per = ceil(ntl / 64) <= R tiles
template <int R>
__device__ void tile_level_w(const Dev &d, int64_t first, int64_t ntl, int64_t lt, double &y_in,
                             double &phi_above, double &dp_top)
{
    const int lane = lane_id();
    const int64_t per = (ntl + 63) / 64;
    const int64_t n_runs = (ntl + per - 1) / per;
    // lane l: forward run l, backward run n_runs - 1 - l
    const int64_t a0 = (int64_t)lane * per;
    const int64_t a1 = min(a0 + per, ntl);
    const int64_t q = n_runs - 1 - (int64_t)lane;
    const int64_t b0 = q >= 0 ? q * per : 0;
    const int64_t b1 = q >= 0 ? min(b0 + per, ntl) : 0;
    const AffineStatus one = {1.0, 0.0};
    const BackStatus bone = {1.0, 0.0, 0.0};
    AffineStatus F[R], FB[R];
    BackStatus B[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        F[i] = (a0 + i < a1) ? d.fwd_status[first + a0 + i] : one;
        FB[i] = (b0 + i < b1) ? d.fwd_status[first + b0 + i] : one;
        B[i] = (b0 + i < b1) ? d.bwd_status[first + b0 + i] : bone;
    }
    // forward: the runs' composites scanned from the bottom up
    Aff m = {1.0, 0.0};
#pragma unroll
    for (int i = 0; i < R; ++i)
        if (a0 + i < a1) m = compose(Aff{F[i].A, F[i].B}, m);
    Aff inc = m;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const Aff o = shfl_up_aff(inc, s);
        if (lane >= s) inc = compose(inc, o);
    }
    Aff ex = shfl_up_aff(inc, 1);
    if (lane == 0) ex = Aff{1.0, 0.0};
    const double y_run = ex.B;  // d' entering this lane's run (d'_0 = 0)
    {
        double y = y_run;
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (a0 + i < lt) y = F[i].A * y + F[i].B;
        y_in = __shfl(y, (int)(lt / per), 64);  // from the lane whose run holds tile lt
    }
    dp_top = __shfl(inc.B, 63, 64);
    // backward: each tile's map with the d' entering it, from the top down
    Aff bk[R];
    {
        double y = __shfl(y_run, (int)(q >= 0 ? q : 0), 64);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            bk[i] = Aff{B[i].A, B[i].B0 + B[i].B1 * y};
            y = FB[i].A * y + FB[i].B;
        }
    }
    Aff mb = {1.0, 0.0};
#pragma unroll
    for (int i = R - 1; i >= 0; --i)
        if (b0 + i < b1) mb = compose(bk[i], mb);
    Aff incb = mb;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const Aff o = shfl_up_aff(incb, s);
        if (lane >= s) incb = compose(incb, o);
    }
    Aff exb = shfl_up_aff(incb, 1);
    if (lane == 0) exb = Aff{1.0, 0.0};
    {
        Aff M = exb;
#pragma unroll
        for (int i = R - 1; i >= 0; --i)
            if (b0 + i < b1 && b0 + i > lt) M = compose(bk[i], M);
        phi_above = __shfl(M.B, (int)(n_runs - 1 - lt / per), 64);  // from the lane whose run holds tile lt
    }
}

// the same for runs of any length, read tile by tile
__device__ void tile_level_any(const Dev &d, int64_t first, int64_t ntl, int64_t lt, double &y_in,
                               double &phi_above, double &dp_top)
{
    __shared__ double s_y[kBlock];  // d' entering each run
    __shared__ double s_out[2];
    const int64_t per = (ntl + kBlock - 1) / kBlock;
    const int64_t n_runs = (ntl + per - 1) / per;
    // d' entering tile t of the run starting at q0 with entering value y
    auto enter = [&](int64_t q0, int64_t t, double y) {
        for (int64_t u = q0; u < t; ++u) {
            const AffineStatus &f = d.fwd_status[first + u];
            y = f.A * y + f.B;
        }
        return y;
    };
    const int64_t a0 = (int64_t)threadIdx.x * per;
    const int64_t a1 = min(a0 + per, ntl);
    Aff m = {1.0, 0.0};
    for (int64_t t = a0; t < a1; ++t) {
        const AffineStatus &f = d.fwd_status[first + t];
        m = compose(Aff{f.A, f.B}, m);
    }
    Aff agg;
    const Aff ex = block_exclusive_scan(m, &agg);
    s_y[threadIdx.x] = ex.B;
    if (a0 <= lt && lt < a1) s_out[0] = enter(a0, lt, ex.B);
    __syncthreads();
    const int64_t q = n_runs - 1 - (int64_t)threadIdx.x;
    int64_t b0 = 0, b1 = 0;
    Aff mb = {1.0, 0.0};
    auto back = [&](int64_t t) {
        const BackStatus &b = d.bwd_status[first + t];
        return Aff{b.A, b.B0 + b.B1 * enter(b0, t, s_y[q])};
    };
    if (q >= 0) {
        b0 = q * per;
        b1 = min(b0 + per, ntl);
        for (int64_t t = b1 - 1; t >= b0; --t) mb = compose(back(t), mb);
    }
    Aff aggb;
    const Aff exb = block_exclusive_scan(mb, &aggb);
    if (q >= 0 && b0 <= lt && lt < b1) {
        Aff M = exb;
        for (int64_t t = b1 - 1; t > lt; --t) M = compose(back(t), M);
        s_out[1] = M.B;
    }
    __syncthreads();
    y_in = s_out[0];
    phi_above = s_out[1];
    dp_top = agg.B;
}

__device__ __forceinline__ void tile_level(const Dev &d, int64_t first, int64_t ntl, int64_t lt, double &y_in,
                                           double &phi_above, double &dp_top)
{
    if (ntl <= 64) tile_level_w<1>(d, first, ntl, lt, y_in, phi_above, dp_top);
    else if (ntl <= 128) tile_level_w<2>(d, first, ntl, lt, y_in, phi_above, dp_top);
    else if (ntl <= 256) tile_level_w<4>(d, first, ntl, lt, y_in, phi_above, dp_top);
    else if (ntl <= (int64_t)kRunR * kBlock) tile_level_r<kRunR>(d, first, ntl, lt, y_in, phi_above, dp_top);
    else tile_level_any(d, first, ntl, lt, y_in, phi_above, dp_top);
}

// ---------------------------------------------------------------------------
// 2. the values entering the tile, d' and phi of its nodes, E, acc,
//    field-energy partials; clears the deposit
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void field_bwd_kernel(Dev d)
{
    const int64_t vt = blockIdx.x;
    const int inst = seg_of_tile(d.inst_ftile0, d.n_inst, vt);
    // the instance's and its species' constants read once, before any store
    // (read after the stores below, the compiler would read them again per
    // node and wait for every store before it)
    const InstConst &ic = d.instc[inst];
    const int64_t ftile0 = ic.ftile0, gnode = ic.gnode;
    const int64_t ntl = d.inst_ftile0[inst + 1] - ftile0;
    const int64_t lt = vt - ftile0;
    const int nc = ic.nc;
    const bool periodic = (ic.bc == PIC_BC_PERIODIC);
    const bool field_off = ic.field_off != 0;
    const int64_t G = d.G;
    const int nsp = ic.nsp;
    const double dx = ic.dx, eps0 = ic.eps0;
    const int64_t lo = lt * kFieldTile;
    double accC[PIC_MAX_SPECIES];  // a species past nsp repeats the last one, unused
#pragma unroll
    for (int k = 0; k < PIC_MAX_SPECIES; ++k) accC[k] = d.segc[ic.seg0 + min(k, nsp - 1)].accC;

    // the thread's nodes (thread t: nodes lo + t kFieldR up): their forward
    // terms and the backward maps of the threads above them, loaded before
    // the first wait, and rho at the walls
    const int64_t c = threadIdx.x;
    const int64_t j0 = lo + c * kFieldR;
    NodeSweep sw[kFieldR];
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) sw[r] = d.sweep[vt * kFieldTile + c * kFieldR + r];
    const BackStatus bp = d.bpre[vt * kBlock + c];
    const double rho_0 = d.rho[gnode], rho_nc = d.rho[gnode + nc];

    double y_in, phi_above, dp_top;
    tile_level(d, ftile0, ntl, lt, y_in, phi_above, dp_top);

    // d' = d0 + h y_in at each node, and phi from the top down, entering the
    // thread's nodes with the maps of the threads above applied to phi_above
    double ph[kFieldR];
    double y = bp.A * phi_above + (bp.B0 + bp.B1 * y_in);
#pragma unroll
    for (int r = kFieldR - 1; r >= 0; --r) {
        const int64_t j = j0 + r;
        if (j >= 1 && j <= nc - 1) {
            y = gq_of(j) * y + (sw[r].d0 + sw[r].h * y_in);
            ph[r] = y;
        } else {
            ph[r] = 0.0;  // nodes 0 and nc (and beyond the grid)
        }
    }
    // neighbours through LDS: s_phi[1 + i] = phi at node lo + i
    __shared__ double s_phi[kFieldTile + 2];
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) s_phi[1 + c * kFieldR + r] = ph[r];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t hi1 = lo + kFieldTile;  // first node above the tile
        s_phi[kFieldTile + 1] = (hi1 <= nc - 1) ? phi_above : 0.0;
        double below = 0.0;                   // phi at node lo - 1 (d' there: the value entering the tile)
        if (lo - 1 >= 1) below = gq_of(lo - 1) * s_phi[1] + y_in;
        s_phi[0] = below;
    }
    __syncthreads();

    double fe = 0.0;
    double phi_nm1 = 0.0;
    if (periodic && lo == 0 && nc >= 2) phi_nm1 = dp_top;  // phi_{nc-1} = d'_{nc-1}
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) {
        const int64_t j = j0 + r;
        if (j > nc) continue;
        const int64_t i = j - lo;
        const double pl = s_phi[i], pc = s_phi[1 + i], pr = s_phi[2 + i];
        double E;
        double V = dx;
        if (j >= 1 && j <= nc - 1) {
            E = (pl - pr) / (2.0 * dx);
        } else if (periodic) {
            // node nc is node 0; gauge phi_0 = 0
            const double p1 = (j == 0) ? pr : 0.0;
            E = (phi_nm1 - p1) / (2.0 * dx);
            if (j == nc) {
                // E_nc = E_0; computed by the tile owning node 0 and copied below
                E = 0.0;
                V = 0.0;
            }
        } else if (j == 0) {
            E = -(pr - pc) / dx - rho_0 * dx / (2.0 * eps0);
            V = 0.5 * dx;
        } else {  // j == nc, absorbing
            E = -(pc - pl) / dx + rho_nc * dx / (2.0 * eps0);
            V = 0.5 * dx;
        }
        if (field_off) E = 0.0;  // no field solve in this instance
        d.phi[gnode + j] = field_off ? 0.0 : pc;
        if (!(periodic && j == nc)) {
            d.E[gnode + j] = E;
            fe += E * E * V;
#pragma unroll
            for (int k = 0; k < PIC_MAX_SPECIES; ++k) {
                if (k >= nsp) break;
                const double a = accC[k] * E;
                d.acc64[k * G + gnode + j] = a;
                d.acc32[k * G + gnode + j] = (float)a;
                if (periodic && j == 0) {
                    d.acc64[k * G + gnode + nc] = a;
                    d.acc32[k * G + gnode + nc] = (float)a;
                }
            }
            if (periodic && j == 0) d.E[gnode + nc] = E;
        }
#pragma unroll
        for (int k = 0; k < PIC_MAX_SPECIES; ++k)
            if (k < nsp) d.S[k * G + gnode + j] = 0ull;
    }
    // field-energy partial of the tile (1/2 eps0 applied by the diagnostics)
    // (a halving tree: the two levels across waves through LDS, the six
    // inside wave 0 through shuffles, the same sums in the same order)
    __shared__ double s_fe[kBlock];
    s_fe[threadIdx.x] = fe;
    __syncthreads();
    static_assert(kBlock == 256, "the levels below are written for 256 threads");
    if (threadIdx.x < 128) s_fe[threadIdx.x] += s_fe[threadIdx.x + 128];
    __syncthreads();
    if (threadIdx.x < 64) {
        double v = s_fe[threadIdx.x] + s_fe[threadIdx.x + 64];
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) {
            const double o = __shfl_down(v, s, 64);
            if (threadIdx.x < s) v += o;
        }
        if (threadIdx.x == 0) d.fe_part[ftile0 + lt] = v;
    }
}

// ---------------------------------------------------------------------------
// density smoother (Sec. 2, phase 2): one pass of the binomial (1,2,1)/4
// filter on the node charges Q_j = rho_j V_j of every instance with more
// than `pass` passes (the others are copied).  The first pass reads rho and
// forms Q, the last divides by V again, so Q is carried between passes as the
// oracle carries it.  At an absorbing wall the outgoing quarter stays on the
// wall node; a periodic grid wraps and node nc repeats node 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void field_smooth_kernel(Dev d, const double *in, double *out,
                                                             int pass, int last_pass)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= d.G) return;
    const int inst = seg_of_tile(d.node_base, d.n_inst, g);
    const InstConst &ic = d.instc[inst];
    const int64_t j = g - ic.gnode;
    const int nc = ic.nc;
    const bool periodic = (ic.bc == PIC_BC_PERIODIC);
    const int passes = ic.field_off ? 0 : ic.smooth_passes;
    if (pass >= passes) {  // not smoothed this pass: carry the value through
        out[g] = in[g];
        return;
    }
    const bool first = (pass == 0), last = (pass == passes - 1) || (pass == last_pass);
    const double dx = ic.dx;
    auto vol = [&](int64_t q) { return (!periodic && (q == 0 || q == nc)) ? 0.5 * dx : dx; };
    auto charge = [&](int64_t q) { return first ? in[ic.gnode + q] * vol(q) : in[ic.gnode + q]; };
    int64_t jj = j, jl, jr;
    if (periodic) {
        if (jj == nc) jj = 0;
        jl = jj > 0 ? jj - 1 : nc - 1;
        jr = jj < nc - 1 ? jj + 1 : 0;
    } else {
        jl = jj > 0 ? jj - 1 : jj;
        jr = jj < nc ? jj + 1 : jj;
    }
    const double r = (charge(jl) + 2.0 * charge(jj) + charge(jr)) * 0.25;
    out[g] = last ? r / vol(jj) : r;
}

hipError_t launch_field(const Dev &d, hipStream_t st, int smooth, int close_mode)
{
    const dim3 grid((unsigned)d.n_field_tiles), block(kBlock);
    // the first launch, with one block more when it closes the step
    const int mode0 = d.field_all_off ? (int)kRhoNoSolve : (int)kRhoSolve;
    if (close_mode >= 0)
        hipLaunchKernelGGL(field_rho_kernel<true>, dim3(grid.x + 1), block, 0, st, d, mode0, close_mode);
    else
        hipLaunchKernelGGL(field_rho_kernel<false>, grid, block, 0, st, d, mode0, -1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || d.field_all_off) return e;
    if (smooth > 0) {
        // passes alternate between rho and the d' array (free until the forward sweep)
        const dim3 ng((unsigned)((d.G + kBlock - 1) / kBlock));
        double *a = d.rho, *b = d.dprime;
        for (int p = 0; p < smooth; ++p) {
            hipLaunchKernelGGL(field_smooth_kernel, ng, block, 0, st, d, a, b, p, smooth - 1);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            double *t = a;
            a = b;
            b = t;
        }
        if (a != d.rho) {  // an odd number of passes: the result is in d'
            hipLaunchKernelGGL(field_smooth_kernel, ng, block, 0, st, d, (const double *)a, d.rho,
                               smooth, smooth);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(field_rho_kernel<false>, grid, block, 0, st, d, (int)kRhoFromRho, -1);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(field_bwd_kernel, grid, block, 0, st, d);
    return hipGetLastError();
}

}  // namespace picx
