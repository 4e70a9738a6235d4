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
// thread composes kFieldR consecutive maps, the block scans the thread maps,
// and tiles chain through a single-pass decoupled look-back in which one wave
// inspects 64 predecessor tiles per round.  Same recurrences
// as the sequential sweep, regrouped; only the rounding order differs.
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

__device__ __forceinline__ void st_release(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Look-back over the tiles before `vt` of the same instance, by the 64 lanes
// of one wave: each round inspects 64 predecessors at once and composes the
// aggregates up to the nearest inclusive one.  Publishes this tile's
// aggregate first and its inclusive value last; returns the value entering
// the tile (in every lane).
__device__ double affine_lookback(AffineStatus *st, int64_t vt, int64_t lt, Aff agg,
                                  unsigned long long gen)
{
    const int lane = lane_id();
    if (lt == 0) {
        if (lane == 0) {
            st[vt].V = agg.B;  // applied to the boundary value 0
            st_release(&st[vt].flag, (gen << 2) | 2ull);
        }
        return 0.0;
    }
    if (lane == 0) {
        st[vt].A = agg.A;
        st[vt].B = agg.B;
        st_release(&st[vt].flag, (gen << 2) | 1ull);
    }
    const int64_t p_first = vt - lt;  // tile 0 of the instance: always inclusive
    Aff R = {1.0, 0.0};               // maps of the closer tiles, applied last
    double y_in = 0.0;
    for (int64_t p_hi = vt - 1;; p_hi -= 64) {
        const int64_t p = p_hi - lane;
        const bool inr = p >= p_first;
        unsigned long long f = 0;
        if (inr) {
            // poll without acquire (an acquire invalidates the L2 on every poll)
            do {
                f = __hip_atomic_load(&st[p].flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } while ((f >> 2) != gen);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const bool incl = inr && ((f & 3ull) == 2ull);
        const unsigned long long mb = ballot(incl);
        const int k = mb ? (__ffsll((long long)mb) - 1) : 64;
        Aff m = {1.0, 0.0};
        if (inr && lane < k) m = Aff{st[p].A, st[p].B};
        // m_0 o m_1 o ... o m_{k-1} (lane 0 is the closest tile)
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            Aff o;
            o.A = __shfl_down(m.A, dd, 64);
            o.B = __shfl_down(m.B, dd, 64);
            if (lane + dd < 64) m = compose(m, o);
        }
        Aff c;
        c.A = __shfl(m.A, 0, 64);
        c.B = __shfl(m.B, 0, 64);
        R = compose(R, c);
        if (mb) {
            double V = 0.0;
            if (lane == k) V = st[p].V;
            V = __shfl(V, k, 64);
            y_in = R.A * V + R.B;
            break;
        }
    }
    if (lane == 0) {
        st[vt].V = agg.A * y_in + agg.B;
        st_release(&st[vt].flag, (gen << 2) | 2ull);
    }
    return y_in;
}

__device__ __forceinline__ void scan_ticket(Globals *g, int id, int64_t *vt, unsigned long long *gen)
{
    __shared__ uint32_t s_t;
    __shared__ unsigned long long s_g;
    if (threadIdx.x == 0) {
        s_g = __hip_atomic_load(&g->scan_gen[id], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_t = atomicAdd(&g->scan_ticket[id], 1u);
    }
    __syncthreads();
    *vt = s_t;
    *gen = s_g;
}

// the last tile to finish resets the ticket counter and advances the generation
__device__ __forceinline__ void scan_finish(Globals *g, int id, int64_t n_tiles)
{
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&g->scan_finish[id], 1u);
        if ((int64_t)prev == n_tiles - 1) {
            g->scan_ticket[id] = 0;
            g->scan_finish[id] = 0;
            g->scan_gen[id] = g->scan_gen[id] + 1ull;
            __threadfence();
        }
    }
}

// ---------------------------------------------------------------------------
// forward sweep: rho, d, d'
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void field_fwd_kernel(Dev d)
{
    int64_t vt;
    unsigned long long gen;
    scan_ticket(d.glob, kScanFwd, &vt, &gen);
    const int inst = seg_of_tile(d.inst_ftile0, d.n_inst, vt);
    const InstConst &ic = d.instc[inst];
    const int64_t lt = vt - ic.ftile0;
    const int nc = ic.nc;
    const bool periodic = (ic.bc == PIC_BC_PERIODIC);
    const int64_t G = d.G;
    const int nsp = ic.nsp;
    const double two_m32 = 0x1p-32;

    // uniform background for periodic systems, from the live counts
    double rho_bg = 0.0;
    if (periodic) {
        double qn = 0.0;
        for (int k = 0; k < nsp; ++k) {
            const SegConst &sc = d.segc[ic.seg0 + k];
            qn += sc.qw * (double)d.segd[ic.seg0 + k].live;
        }
        rho_bg = -qn / ((double)nc * ic.dx);
    }

    const int64_t j0 = lt * kFieldTile + (int64_t)threadIdx.x * kFieldR;
    double dv[kFieldR];
    Aff m = {1.0, 0.0};
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) {
        const int64_t j = j0 + r;
        dv[r] = 0.0;
        if (j <= nc) {
            double acc = 0.0;
            for (int k = 0; k < nsp; ++k) {
                const unsigned long long *S = d.S + k * G + ic.gnode;
                unsigned long long Sj = S[j];
                if (periodic) {
                    if (j == 0) Sj += S[nc];
                    if (j == nc) Sj = S[0] + S[nc];
                }
                acc += d.segc[ic.seg0 + k].qw * ((double)Sj * two_m32);
            }
            double V = ic.dx;
            if (!periodic && (j == 0 || j == nc)) V = 0.5 * ic.dx;
            const double rho = acc / V + rho_bg;
            d.rho[ic.gnode + j] = rho;
            if (j >= 1 && j <= nc - 1) {
                const double dd = -(rho * ic.K);
                const double u = (double)j;
                const double gq = u / (u + 1.0);  // -g_u
                dv[r] = dd;
                m = compose(Aff{gq, -(gq * dd)}, m);
            }
        }
    }
    Aff agg;
    const Aff excl = block_exclusive_scan(m, &agg);
    __shared__ double s_in;
    if (threadIdx.x < 64) {
        const double y = affine_lookback(d.fwd_status, vt, lt, agg, gen);
        if (threadIdx.x == 0) s_in = y;
    }
    __syncthreads();
    double y = excl.A * s_in + excl.B;
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) {
        const int64_t j = j0 + r;
        if (j >= 1 && j <= nc - 1) {
            const double u = (double)j;
            const double gq = u / (u + 1.0);
            y = gq * y + (-(gq * dv[r]));
            d.dprime[ic.gnode + j] = y;
        }
    }
    scan_finish(d.glob, kScanFwd, d.n_field_tiles);
}

// ---------------------------------------------------------------------------
// backward sweep: phi, E, acc, field-energy partials; clears the deposit
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void field_bwd_kernel(Dev d)
{
    int64_t vt_r;
    unsigned long long gen;
    scan_ticket(d.glob, kScanBwd, &vt_r, &gen);
    // tickets run from the top tile of each instance down
    const int inst = seg_of_tile(d.inst_ftile0, d.n_inst, vt_r);
    const InstConst &ic = d.instc[inst];
    const int64_t ntl = d.inst_ftile0[inst + 1] - ic.ftile0;
    const int64_t lt_r = vt_r - ic.ftile0;        // 0 = top tile
    const int64_t lt = ntl - 1 - lt_r;            // node tile index
    const int nc = ic.nc;
    const bool periodic = (ic.bc == PIC_BC_PERIODIC);
    const int64_t G = d.G;
    const int nsp = ic.nsp;
    const double dx = ic.dx;

    // thread t owns the chunk counted from the top of the tile
    const int64_t lo = lt * kFieldTile;
    const int64_t c = kBlock - 1 - threadIdx.x;
    const int64_t j0 = lo + c * kFieldR;
    double dp[kFieldR];
    Aff m = {1.0, 0.0};
#pragma unroll
    for (int r = kFieldR - 1; r >= 0; --r) {
        const int64_t j = j0 + r;
        dp[r] = 0.0;
        if (j >= 1 && j <= nc - 1) {
            dp[r] = d.dprime[ic.gnode + j];
            const double u = (double)j;
            m = compose(Aff{u / (u + 1.0), dp[r]}, m);
        }
    }
    Aff agg;
    const Aff excl = block_exclusive_scan(m, &agg);
    __shared__ double s_in;
    if (threadIdx.x < 64) {
        const double y = affine_lookback(d.bwd_status, vt_r, lt_r, agg, gen);
        if (threadIdx.x == 0) s_in = y;
    }
    __syncthreads();
    const double phi_above = s_in;  // phi at the node just above this tile (0 at the top)

    // phi for the thread's nodes, top down
    double ph[kFieldR];
    double y = excl.A * phi_above + excl.B;
#pragma unroll
    for (int r = kFieldR - 1; r >= 0; --r) {
        const int64_t j = j0 + r;
        if (j >= 1 && j <= nc - 1) {
            const double u = (double)j;
            y = (u / (u + 1.0)) * y + dp[r];
            ph[r] = y;
        } else {
            ph[r] = 0.0;  // nodes 0 and nc (and beyond the grid)
        }
    }
    // neighbours through LDS: s_phi[1 + i] = phi at node lo + i
    __shared__ double s_phi[kFieldTile + 2];
#pragma unroll
    for (int r = 0; r < kFieldR; ++r) s_phi[1 + c * kFieldR + r] = ph[r];
    if (threadIdx.x == 0) {
        const int64_t hi1 = lo + kFieldTile;  // first node above the tile
        s_phi[kFieldTile + 1] = (hi1 <= nc - 1) ? phi_above : 0.0;
        double below = 0.0;                   // phi at node lo - 1
        if (lo - 1 >= 1) {
            const double u = (double)(lo - 1);
            below = (u / (u + 1.0)) * s_phi[1] + d.dprime[ic.gnode + lo - 1];
        }
        s_phi[0] = below;
    }
    __syncthreads();
    // s_phi[1 + 0] is written by the thread owning chunk 0 before the barrier;
    // recompute `below` after it if thread 0 did not own chunk 0
    if (threadIdx.x == 0 && lo - 1 >= 1) {
        const double u = (double)(lo - 1);
        s_phi[0] = (u / (u + 1.0)) * s_phi[1] + d.dprime[ic.gnode + lo - 1];
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
        d.phi[ic.gnode + j] = pc;
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
    __shared__ double s_fe[kBlock];
    s_fe[threadIdx.x] = fe;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) s_fe[threadIdx.x] += s_fe[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) d.fe_part[ic.ftile0 + lt] = s_fe[0];
    scan_finish(d.glob, kScanBwd, d.n_field_tiles);
}

hipError_t launch_field(const Dev &d, hipStream_t st)
{
    const dim3 grid((unsigned)d.n_field_tiles), block(kBlock);
    hipLaunchKernelGGL(field_fwd_kernel, grid, block, 0, st, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(field_bwd_kernel, grid, block, 0, st, d);
    return hipGetLastError();
}

}  // namespace picx
