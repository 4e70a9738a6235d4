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
// maps.  Tiles chain through three launches, with no atomics and no waiting
// between blocks:
//   1. rho, and the composite of each tile's forward maps;
//   2. the composites of the tiles below give the value entering the tile;
//      forward sweep (d'), and the composite of the tile's backward maps;
//   3. the composites of the tiles above give phi entering the tile from the
//      top; backward sweep (phi), then E, the accelerations, the field energy.
// Same recurrences as the sequential sweep, regrouped; only the rounding
// order differs.
//
// The first launch also forms the node density of a kinetic neutral species,
//   n_j = w_n S_n[j] 2^-32 / V_j,
// which the collisions gather at the electrons.  An instance without a field
// solve (the paper's Table 1 case) gets E = phi = 0; when no instance solves
// the field, the first launch alone runs (rho, the neutral density, the
// deposit cleared).
#include "device_common.h"

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

// Composite of n maps taken in application order a = 0..n-1, where map a is
// agg[idx(a)]: every thread composes a contiguous run, then an ordered tree
// over the block.  Returns the composite in every thread.
template <class Idx>
__device__ Aff compose_ordered(const AffineStatus *agg, int64_t n, Idx idx)
{
    __shared__ Aff s_m[kWaves];
    const int64_t per = (n + kBlock - 1) / kBlock;
    const int64_t a0 = (int64_t)threadIdx.x * per;
    Aff m = {1.0, 0.0};
    for (int64_t a = a0; a < a0 + per && a < n; ++a) {
        const AffineStatus &s = agg[idx(a)];
        m = compose(Aff{s.A, s.B}, m);
    }
    // the tree's levels inside a wave through shuffles (the same pairs in the
    // same order as a tree over LDS, without a barrier per level), then the
    // four wave composites
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const Aff o = {__shfl_down(m.A, s, 64), __shfl_down(m.B, s, 64)};
        if ((lane & (2 * s - 1)) == 0) m = compose(o, m);
    }
    static_assert(kWaves == 4, "the cross-wave levels below are written for four waves");
    if (lane == 0) s_m[wave] = m;
    __syncthreads();
    const Aff r = compose(compose(s_m[3], s_m[2]), compose(s_m[1], s_m[0]));
    __syncthreads();
    return r;
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
// no composites (no instance solves the field)
__global__ __launch_bounds__(kBlock) void field_rho_kernel(Dev d, int mode)
{
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
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) {
        const int64_t j = j0 + r;
        if (j > nc) continue;
        if (from_rho) {
            if (j >= 1 && j <= nc - 1) {
                const double dd = -(d.rho[gnode + j] * K);
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
    (void)block_exclusive_scan(m, &agg);
    if (threadIdx.x == 0) {
        d.fwd_status[vt].A = agg.A;
        d.fwd_status[vt].B = agg.B;
    }
}

// ---------------------------------------------------------------------------
// 2. forward sweep (d') and the backward composite of every tile
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void field_fwd_kernel(Dev d)
{
    const int64_t vt = blockIdx.x;
    const int inst = seg_of_tile(d.inst_ftile0, d.n_inst, vt);
    const InstConst &ic = d.instc[inst];
    const int64_t lt = vt - ic.ftile0;
    const int nc = ic.nc;

    // the thread's rho, loaded before the first wait (unpredicated: a node
    // past nc reads node nc and is not used)
    const int64_t j0 = lt * kFieldTile + (int64_t)threadIdx.x * kFieldR;
    double rl[kFieldR];
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) rl[r] = d.rho[ic.gnode + min(j0 + r, (int64_t)nc)];

    // d' entering the tile: the composites of the tiles below applied to d'_0 = 0
    const int64_t first = ic.ftile0;
    const Aff below = compose_ordered(d.fwd_status, lt, [first](int64_t a) { return first + a; });

    double dv[kFieldR];
    Aff m = {1.0, 0.0};
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) {
        const int64_t j = j0 + r;
        dv[r] = 0.0;
        if (j >= 1 && j <= nc - 1) {
            dv[r] = -(rl[r] * ic.K);
            const double gq = gq_of(j);
            m = compose(Aff{gq, -(gq * dv[r])}, m);
        }
    }
    Aff agg;
    const Aff excl = block_exclusive_scan(m, &agg);
    double y = excl.A * below.B + excl.B;
    double dp[kFieldR];
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) {
        const int64_t j = j0 + r;
        dp[r] = 0.0;
        if (j >= 1 && j <= nc - 1) {
            const double gq = gq_of(j);
            y = gq * y + (-(gq * dv[r]));
            d.dprime[ic.gnode + j] = y;
            dp[r] = y;
        }
    }
    // backward maps phi_u = (u/(u+1)) phi_{u+1} + d'_u of the thread's nodes, top first
    Aff mb = {1.0, 0.0};
#pragma unroll
    for (int r = kFieldR - 1; r >= 0; --r) {
        const int64_t j = j0 + r;
        if (j >= 1 && j <= nc - 1) mb = compose(Aff{gq_of(j), dp[r]}, mb);
    }
    // the block's composite: threads from the top down, i.e. an ordered tree
    // over i = kBlock - 1 - thread.  Inside a wave index i is lane 63 - l of
    // group 3 - wave, so each level takes the lane s below (the same pairs in
    // the same order as the tree over LDS, without a barrier per level).
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const Aff o = shfl_up_aff(mb, s);
        if (((63 - lane) & (2 * s - 1)) == 0) mb = compose(o, mb);
    }
    static_assert(kWaves == 4, "the cross-wave levels below are written for four waves");
    __shared__ Aff s_b[kWaves];
    if (lane == 63) s_b[wave] = mb;  // the composite of group 3 - wave
    __syncthreads();
    if (threadIdx.x == 0) {
        const Aff r = compose(compose(s_b[0], s_b[1]), compose(s_b[2], s_b[3]));
        d.bwd_status[vt].A = r.A;
        d.bwd_status[vt].B = r.B;
    }
}

// ---------------------------------------------------------------------------
// 3. backward sweep: phi, E, acc, field-energy partials; clears the deposit
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void field_bwd_kernel(Dev d)
{
    const int64_t vt = blockIdx.x;
    const int inst = seg_of_tile(d.inst_ftile0, d.n_inst, vt);
    const InstConst &ic = d.instc[inst];
    const int64_t ntl = d.inst_ftile0[inst + 1] - ic.ftile0;
    const int64_t lt = vt - ic.ftile0;
    const int nc = ic.nc;
    const bool periodic = (ic.bc == PIC_BC_PERIODIC);
    const int64_t G = d.G;
    const int nsp = ic.nsp;
    const double dx = ic.dx;

    // thread t owns the chunk counted from the top of the tile; its d' is
    // loaded before the first wait (unpredicated: a node past nc reads node
    // nc and is not used)
    const int64_t lo = lt * kFieldTile;
    const int64_t c = kBlock - 1 - threadIdx.x;
    const int64_t j0 = lo + c * kFieldR;
    double dl[kFieldR];
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) dl[r] = d.dprime[ic.gnode + min(j0 + r, (int64_t)nc)];

    // phi at the first node above the tile: the composites of the tiles
    // above, top first, applied to phi_nc = 0
    const int64_t last = ic.ftile0 + ntl - 1;
    const Aff above = compose_ordered(d.bwd_status, ntl - 1 - lt, [last](int64_t a) { return last - a; });
    const double phi_above = above.B;

    double dp[kFieldR];
    Aff m = {1.0, 0.0};
#pragma unroll
    for (int r = kFieldR - 1; r >= 0; --r) {
        const int64_t j = j0 + r;
        dp[r] = 0.0;
        if (j >= 1 && j <= nc - 1) {
            dp[r] = dl[r];
            m = compose(Aff{gq_of(j), dp[r]}, m);
        }
    }
    Aff agg;
    const Aff excl = block_exclusive_scan(m, &agg);

    // phi for the thread's nodes, top down
    double ph[kFieldR];
    double y = excl.A * phi_above + excl.B;
#pragma unroll
    for (int r = kFieldR - 1; r >= 0; --r) {
        const int64_t j = j0 + r;
        if (j >= 1 && j <= nc - 1) {
            y = gq_of(j) * y + dp[r];
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
        double below = 0.0;                   // phi at node lo - 1
        if (lo - 1 >= 1) below = gq_of(lo - 1) * s_phi[1] + d.dprime[ic.gnode + lo - 1];
        s_phi[0] = below;
    }
    __syncthreads();

    double fe = 0.0;
    double phi_nm1 = 0.0;
    if (periodic && lo == 0 && nc >= 2) phi_nm1 = d.dprime[ic.gnode + nc - 1];  // phi_{nc-1} = d'_{nc-1}
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
            E = -(pr - pc) / dx - d.rho[ic.gnode] * dx / (2.0 * ic.eps0);
            V = 0.5 * dx;
        } else {  // j == nc, absorbing
            E = -(pc - pl) / dx + d.rho[ic.gnode + nc] * dx / (2.0 * ic.eps0);
            V = 0.5 * dx;
        }
        if (ic.field_off) E = 0.0;  // no field solve in this instance
        d.phi[ic.gnode + j] = ic.field_off ? 0.0 : pc;
        if (!(periodic && j == nc)) {
            d.E[ic.gnode + j] = E;
            fe += E * E * V;
            for (int k = 0; k < nsp; ++k) {
                const double a = d.segc[ic.seg0 + k].accC * E;
                d.acc64[k * G + ic.gnode + j] = a;
                d.acc32[k * G + ic.gnode + j] = (float)a;
                if (periodic && j == 0) {
                    d.acc64[k * G + ic.gnode + nc] = a;
                    d.acc32[k * G + ic.gnode + nc] = (float)a;
                }
            }
            if (periodic && j == 0) d.E[ic.gnode + nc] = E;
        }
        for (int k = 0; k < nsp; ++k) d.S[k * G + ic.gnode + j] = 0ull;
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
        if (threadIdx.x == 0) d.fe_part[ic.ftile0 + lt] = v;
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

hipError_t launch_field(const Dev &d, hipStream_t st, int smooth)
{
    const dim3 grid((unsigned)d.n_field_tiles), block(kBlock);
    if (d.field_all_off) {
        hipLaunchKernelGGL(field_rho_kernel, grid, block, 0, st, d, (int)kRhoNoSolve);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(field_rho_kernel, grid, block, 0, st, d, (int)kRhoSolve);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
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
        hipLaunchKernelGGL(field_rho_kernel, grid, block, 0, st, d, (int)kRhoFromRho);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(field_fwd_kernel, grid, block, 0, st, d);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(field_bwd_kernel, grid, block, 0, st, d);
    return hipGetLastError();
}

}  // namespace picx
