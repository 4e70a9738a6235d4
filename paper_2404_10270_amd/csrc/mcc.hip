// mcc.hip -- collisions and plasma-wall bookkeeping (paper Sec. 2, phase 4:
// Monte Carlo collisions and ionisation, plasma-wall interaction) on gfx950.
//
// Null-collision Monte Carlo (Vahedi & Surendra, CPC 87, 1995) against a
// uniform neutral gas.  The push kernel already tested every particle with
// one Philox block keyed by (id, step) and listed the candidates; here each
// candidate redraws that block, picks a process from r = U(u1) nu_max against
// the cumulative n_n sigma |v| (squared comparisons, FP64), and applies
//   elastic e-n   cold neutral of mass M, isotropic in the centre of mass;
//   charge exch.  the ion takes a neutral's Maxwellian velocity (T_n);
//   ionisation    energy above threshold split U : 1-U between two isotropic
//                 electrons, the new ion Maxwellian at T_n, pair at the parent.
// The emit kernel then creates the ionisation pairs (ids ranked by parent id)
// and the source pairs (as many as ions reached the walls this step), deposits
// them, and its last block closes the step: counts, ids, step index.
#include "device_common.h"

#pragma clang fp contract(off)

namespace picx {

__device__ __forceinline__ double ld_v(const void *p, int64_t g, bool f64)
{
    return f64 ? ((const double *)p)[g] : (double)((const float *)p)[g];
}

__device__ __forceinline__ void st_v(void *p, int64_t g, double v, bool f64)
{
    if (f64) ((double *)p)[g] = v;
    else ((float *)p)[g] = (float)v;
}

__global__ __launch_bounds__(kBlock) void collide_kernel(Dev d)
{
    const int cur = d.glob->cur_set;
    const bool f64 = (d.precision == PIC_FP64);
    uint32_t n = d.glob->cand_count;
    if (n > (uint32_t)d.cand_cap) n = (uint32_t)d.cand_cap;
    const uint32_t stride = gridDim.x * kBlock;
    // uniform trip count so that whole waves take part in the aggregations
    const uint32_t n_round = ((n + stride - 1) / stride) * stride;
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < n_round; c += stride) {
        const bool own = c < n;
        int inst = -1;
        unsigned long long cnt = 0;  // packed counts: cand | el<<12 | iz<<24 | cx<<36 | over<<48
        bool iz = false;
        IzEvent ev;
        if (own) {
            const int64_t g = d.cand[c];
            const int seg = seg_of_slot(d.seg_base, d.n_seg, g);
            const SegConst &sc = d.segc[seg];
            inst = sc.inst;
            const long long step = d.instd[inst].step;
            const unsigned long long pid = d.id[cur][g];
            const double vx = ld_v(d.vx[cur], g, f64);
            const double vy = ld_v(d.vy[cur], g, f64);
            const double vz = ld_v(d.vz[cur], g, f64);
            const uint4 u = draw(pid, step, 0, sc.key0, sc.key1);
            const double v2 = (vx * vx + vy * vy) + vz * vz;
            cnt = 1ull;
            if (v2 > sc.vcap2) cnt += 1ull << 48;
            const double r = u01(u.y) * sc.nu_max;
            const double r2 = r * r;
            if (sc.kind == PIC_KIND_ELECTRON) {
                if (r2 < sc.C0 * v2) {
                    double d0, d1, d2;
                    iso_dir(u.z, u.w, d0, d1, d2);
                    const double gg = sqrt(v2);
                    st_v(d.vx[cur], g, sc.am * vx + sc.bm * gg * d0, f64);
                    st_v(d.vy[cur], g, sc.am * vy + sc.bm * gg * d1, f64);
                    st_v(d.vz[cur], g, sc.am * vz + sc.bm * gg * d2, f64);
                    cnt += 1ull << 12;
                } else if (v2 >= sc.v2_iz && r2 < sc.C1 * v2) {
                    const uint4 u1 = draw(pid, step, 1, sc.key0, sc.key1);
                    const double e_tot = 0.5 * v2 - sc.eps_iz;
                    const double e1 = u01(u.z) * e_tot;
                    const double e2 = e_tot - e1;
                    const double g1 = sqrt(2.0 * e1);
                    double d0, d1, d2;
                    iso_dir(u1.x, u1.y, d0, d1, d2);
                    st_v(d.vx[cur], g, g1 * d0, f64);
                    st_v(d.vy[cur], g, g1 * d1, f64);
                    st_v(d.vz[cur], g, g1 * d2, f64);
                    iz = true;
                    ev.parent_id = pid;
                    ev.slot = (uint32_t)g;
                    ev.seg = seg;
                    ev.g2 = sqrt(2.0 * e2);
                    cnt += 1ull << 24;
                }
            } else {
                if (r2 < sc.C0 * v2) {
                    const uint4 u1 = draw(pid, step, 1, sc.key0, sc.key1);
                    double n0, n1, n2, n3;
                    box_muller(u.z, u.w, n0, n1);
                    box_muller(u1.x, u1.y, n2, n3);
                    st_v(d.vx[cur], g, sc.sig_n * n0, f64);
                    st_v(d.vy[cur], g, sc.sig_n * n1, f64);
                    st_v(d.vz[cur], g, sc.sig_n * n2, f64);
                    cnt += 1ull << 36;
                }
            }
        }
        // ionisation events
        const uint32_t idx = wave_append(&d.glob->ev_count, iz);
        if (iz) {
            if (idx < (uint32_t)d.ev_cap) {
                d.ev[idx] = ev;
                atomicAdd(&d.instd[inst].n_iz_step, 1u);
            } else {
                atomicOr(&d.instd[inst].status, PIC_ST_CANDIDATES);
            }
        }
        // per-instance process counters, summed over runs of equal instance
        bool tail;
        const unsigned long long t = run_sum(inst, cnt, tail);
        if (tail && inst >= 0) {
            InstDyn *idn = d.instd + inst;
            const unsigned long long m12 = 0xFFFull;
            if (t & m12) atomicAdd(&idn->n_candidates, t & m12);
            if ((t >> 12) & m12) atomicAdd(&idn->n_elastic, (t >> 12) & m12);
            if ((t >> 24) & m12) atomicAdd(&idn->n_ionize, (t >> 24) & m12);
            if ((t >> 36) & m12) atomicAdd(&idn->n_cx, (t >> 36) & m12);
            if ((t >> 48) & m12) atomicAdd(&idn->n_over_cap, (t >> 48) & m12);
        }
    }
}

// write one created particle into segment `seg`, in-segment index `i`;
// returns false if it did not fit
__device__ __forceinline__ bool place(const Dev &d, int cur, bool f64, int seg, int64_t i,
                                      unsigned long long id, bool split, int32_t cell, float f,
                                      double x, double vx, double vy, double vz)
{
    const SegConst &sc = d.segc[seg];
    if (i >= (int64_t)sc.cap) {
        atomicOr(&d.instd[sc.inst].status, PIC_ST_CAPACITY);
        return false;
    }
    const int64_t g = sc.base + i;
    unsigned long long *S = d.S + sc.sp * d.G + sc.gnode;
    int j;
    unsigned long long w1;
    if (f64) {
        ((double *)d.x[cur])[g] = x;
        const double jn = floor(x);
        j = (int)jn;
        w1 = (unsigned long long)rint(ldexp(x - jn, PIC_FRAC_BITS));
    } else {
        (void)split;
        ((float *)d.x[cur])[g] = f;
        d.cell[cur][g] = cell;
        j = cell;
        w1 = (unsigned long long)rintf(f * 4294967296.0f);
    }
    st_v(d.vx[cur], g, vx, f64);
    st_v(d.vy[cur], g, vy, f64);
    st_v(d.vz[cur], g, vz, f64);
    d.id[cur][g] = id;
    atomicAdd(S + j, (1ull << PIC_FRAC_BITS) - w1);
    atomicAdd(S + j + 1, w1);
    atomicAdd(&d.segd[seg].created_step, 1u);
    return true;
}

constexpr int kMaxInstLds = 4096;

__global__ __launch_bounds__(kBlock) void emit_kernel(Dev d)
{
    const int cur = d.glob->cur_set;
    const bool f64 = (d.precision == PIC_FP64);
    uint32_t m_all = d.glob->ev_count;
    if (m_all > (uint32_t)d.ev_cap) m_all = (uint32_t)d.ev_cap;
    const uint32_t stride = gridDim.x * kBlock;

    // ---- ionisation pairs: rank each event among its instance's events by parent id
    __shared__ unsigned long long s_pid[kBlock];
    __shared__ int s_inst[kBlock];
    for (uint32_t base = blockIdx.x * kBlock; base < m_all; base += stride) {
        const uint32_t e = base + threadIdx.x;
        const bool own = e < m_all;
        IzEvent ev = {};
        int my_inst = -1;
        if (own) {
            ev = d.ev[e];
            my_inst = d.segc[ev.seg].inst;
        }
        uint32_t rank = 0;
        for (uint32_t cb = 0; cb < m_all; cb += kBlock) {
            __syncthreads();
            const uint32_t k = cb + threadIdx.x;
            if (k < m_all) {
                const IzEvent o = d.ev[k];
                s_pid[threadIdx.x] = o.parent_id;
                s_inst[threadIdx.x] = d.segc[o.seg].inst;
            } else {
                s_pid[threadIdx.x] = ~0ull;
                s_inst[threadIdx.x] = -2;
            }
            __syncthreads();
            if (own) {
                const int lim = (m_all - cb < (uint32_t)kBlock) ? (int)(m_all - cb) : kBlock;
                for (int q = 0; q < lim; ++q)
                    rank += (s_inst[q] == my_inst && s_pid[q] < ev.parent_id) ? 1u : 0u;
            }
        }
        if (own) {
            const SegConst &se = d.segc[ev.seg];
            const int seg_i = se.partner;
            const SegConst &si = d.segc[seg_i];
            const InstDyn &idn = d.instd[se.inst];
            const long long step = idn.step;
            const unsigned long long nid = idn.next_id + 2ull * rank;
            const uint4 u1 = draw(ev.parent_id, step, 1, se.key0, se.key1);
            const uint4 u2 = draw(ev.parent_id, step, 2, se.key0, se.key1);
            double d0, d1, d2;
            iso_dir(u1.z, u1.w, d0, d1, d2);
            double n0, n1, n2, n3;
            box_muller(u2.x, u2.y, n0, n1);
            box_muller(u2.z, u2.w, n2, n3);
            // position of the parent (unchanged by the collision)
            int32_t cell = 0;
            float f = 0.f;
            double x = 0.0;
            if (f64) x = ((const double *)d.x[cur])[ev.slot];
            else {
                cell = d.cell[cur][ev.slot];
                f = ((const float *)d.x[cur])[ev.slot];
            }
            place(d, cur, f64, ev.seg, (int64_t)d.segd[ev.seg].count + rank, nid, false, cell, f, x,
                  ev.g2 * d0, ev.g2 * d1, ev.g2 * d2);
            place(d, cur, f64, seg_i, (int64_t)d.segd[seg_i].count + rank, nid + 1ull, false, cell,
                  f, x, si.sig_n * n0, si.sig_n * n1, si.sig_n * n2);
        }
    }

    // ---- source pairs: instance i creates as many pairs as ions it lost this step
    __shared__ uint32_t s_pre[kMaxInstLds + 1];
    const int n_inst = d.n_inst < kMaxInstLds ? d.n_inst : kMaxInstLds;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int i = 0; i < n_inst; ++i) {
            s_pre[i] = acc;
            const InstConst &ic = d.instc[i];
            if (ic.source_on && ic.seg_i >= 0)
                acc += d.segd[ic.seg_i].absorbed_step[0] + d.segd[ic.seg_i].absorbed_step[1];
        }
        s_pre[n_inst] = acc;
    }
    __syncthreads();
    const uint32_t n_src_all = s_pre[n_inst];
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < n_src_all; q += stride) {
        int lo = 0, hi = n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pre[mid] <= q) lo = mid; else hi = mid - 1;
        }
        const int i = lo;
        const uint32_t k = q - s_pre[i];
        const InstConst &ic = d.instc[i];
        const InstDyn &idn = d.instd[i];
        const SegConst &se = d.segc[ic.seg_e];
        const SegConst &si = d.segc[ic.seg_i];
        const long long step = idn.step;
        const uint32_t m_i = idn.n_iz_step;
        const uint4 b0 = draw_source(k, step, 0, se.key0, se.key1);
        const uint4 b1 = draw_source(k, step, 1, se.key0, se.key1);
        const uint4 b2 = draw_source(k, step, 2, se.key0, se.key1);
        const double x = u01(b0.x) * (double)ic.nc;
        double e0, e1, e2, e3, i0, i1, i2, i3;
        box_muller(b0.y, b0.z, e0, e1);
        box_muller(b1.x, b1.y, e2, e3);
        box_muller(b1.z, b1.w, i0, i1);
        box_muller(b2.x, b2.y, i2, i3);
        int32_t cell = 0;
        float f = 0.f;
        if (!f64) split_position(x, ic.nc, cell, f);
        const unsigned long long nid = idn.next_id + 2ull * (m_i + k);
        place(d, cur, f64, ic.seg_e, (int64_t)d.segd[ic.seg_e].count + m_i + k, nid, true, cell, f,
              x, se.sig_src * e0, se.sig_src * e1, se.sig_src * e2);
        place(d, cur, f64, ic.seg_i, (int64_t)d.segd[ic.seg_i].count + m_i + k, nid + 1ull, true,
              cell, f, x, si.sig_src * i0, si.sig_src * i1, si.sig_src * i2);
    }

    // ---- close of the step, by the last block to finish
    __shared__ bool s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&d.glob->emit_done, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    for (int i = threadIdx.x; i < d.n_inst; i += kBlock) {
        const InstConst &ic = d.instc[i];
        InstDyn *idn = d.instd + i;
        uint32_t n_src = 0;
        if (ic.source_on && ic.seg_i >= 0)
            n_src = d.segd[ic.seg_i].absorbed_step[0] + d.segd[ic.seg_i].absorbed_step[1];
        const uint32_t m_i = idn->n_iz_step;
        unsigned long long pushed = 0;
        for (int k = 0; k < ic.nsp; ++k) {
            const int s = ic.seg0 + k;
            SegDyn *sd = d.segd + s;
            const SegConst &sc = d.segc[s];
            pushed += sd->live;
            uint32_t requested = 0;
            if (s == ic.seg_e || s == ic.seg_i) requested = m_i + n_src;
            uint64_t nc_ = (uint64_t)sd->count + requested;
            if (nc_ > sc.cap) nc_ = sc.cap;
            const uint32_t created = sd->created_step;
            const uint32_t lost = sd->absorbed_step[0] + sd->absorbed_step[1];
            sd->count = (uint32_t)nc_;
            sd->live = sd->live - lost + created;
            sd->absorbed_total[0] += sd->absorbed_step[0];
            sd->absorbed_total[1] += sd->absorbed_step[1];
            sd->created_total += created;
            sd->absorbed_step[0] = 0;
            sd->absorbed_step[1] = 0;
            sd->created_step = 0;
        }
        idn->particle_steps += pushed;
        idn->next_id += 2ull * (unsigned long long)(m_i + n_src);
        idn->n_source += n_src;
        idn->n_iz_step = 0;
        idn->step += 1;
    }
    if (threadIdx.x == 0) {
        d.glob->cand_count = 0;
        d.glob->ev_count = 0;
        d.glob->emit_done = 0;
    }
}

hipError_t launch_collide(const Dev &d, hipStream_t st)
{
    hipLaunchKernelGGL(collide_kernel, dim3(kCollideBlocks), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_emit(const Dev &d, hipStream_t st)
{
    hipLaunchKernelGGL(emit_kernel, dim3(kEmitBlocks), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

}  // namespace picx
