// mcc.hip -- collisions and plasma-wall bookkeeping (paper Sec. 2, phase 4:
// Monte Carlo collisions and ionisation, plasma-wall interaction) on gfx950.
//
// Null-collision Monte Carlo (Vahedi & Surendra, CPC 87, 1995) against a
// uniform neutral gas, or against kinetic neutral atoms (the paper's Table 1
// case, Sec. 3.4).  The push kernel already tested every particle with one
// Philox block keyed by (id, step) and listed the candidates with their
// velocities and ids; here each candidate redraws that block (collide_vel),
// picks a process from r = U(u1) nu_max against the cumulative n sigma |v|
// (squared comparisons, FP64; n is the gas density or the atom density
// gathered at the electron), and applies
//   elastic e-n   cold neutral of mass M, isotropic in the centre of mass;
//   excitation    the electron loses E_ex and leaves isotropically;
//   charge exch.  the ion takes a neutral's Maxwellian velocity (T_n);
//   ionisation    energy above threshold split U : 1-U between two isotropic
//                 electrons; the new ion is Maxwellian at T_n at the parent,
//                 or, with kinetic neutrals, a consumed atom of the parent's
//                 cell (the target kernel picks it).
// The emit kernel then creates the ionisation pairs (ids ranked by parent id)
// and the source pairs (as many as ions reached the walls this step) and
// deposits them; one block closes the step (counts, ids, step index): a
// kernel of its own, or, in a whole step with no periodic instance, one more
// block of the field solve's first launch (step_close.h).
//
// Same-address device atomics from many blocks serialise, so: collide block b
// reads the candidates push block b wrote, writes its ionisation events to its
// own region and keeps its process counts in its own slot.  Readers of the
// events index the regions through a prefix sum built in LDS.
#include "collide_common.h"
#include "step_close.h"

#pragma clang fp contract(off)

namespace picx {

// one block, once per step after the collisions of a batch: the prefix over
// the regions and the totals, for every kernel after it.  (A kernel of its own: folding
// it into the collide kernel's last block costs a device-scope fence in every
// block, which writes back L2 and is far slower than the launch.)
__global__ __launch_bounds__(kBlock) void index_kernel(Dev d)
{
    __shared__ EventIndex X;
    build_event_index(X, d);
    for (int b = threadIdx.x; b <= d.n_push_blocks; b += kBlock) d.ev_pre[b] = X.pre[b];
    if (threadIdx.x == 0) {
        d.glob->ev_total = X.total;
        d.glob->ev_in_regions = X.in_regions;
    }
}

__device__ __forceinline__ const IzEvent &event_at(const EventIndex &X, const Dev &d, uint32_t e)
{
    if (e >= X.in_regions)
        return d.ev[(int64_t)d.n_regions * d.ev_q + (e - X.in_regions)];
    int lo = 0, hi = d.n_push_blocks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (X.pre[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return d.ev[(int64_t)lo * d.ev_q + (e - X.pre[lo])];
}

// The collisions of the listed candidates: block b takes push block b's
// region and a share of the overflow list; OVF_ONLY: only the overflow list
// (after movers that collided their own regions), events to the event
// overflow list.
template <bool SEGLDS, bool OVF_ONLY>
__global__ __launch_bounds__(kBlock) void collide_kernel(Dev d)
{
    extern __shared__ uint32_t s_cnt[];  // [n_seg][kNCnt] when n_seg <= kCntSegMax
    __shared__ uint32_t s_en;
    __shared__ SegConst s_sc[SEGLDS ? kCollSegLds : 1];
    __shared__ long long s_step[SEGLDS ? kCollSegLds : 1];
    if (OVF_ONLY && d.glob->cand_ovf == 0u) return;  // uniform: nothing overflowed this step
    collide_block<SEGLDS>(d, blockIdx.x, !OVF_ONLY, true, nullptr, s_cnt, d.n_seg <= kCntSegMax, s_en,
                          s_sc, s_step);
}

// write one created particle into segment `seg`, in-segment index `i`
// (ignored, and flagged, when the segment is full)
// what placing a created particle in a segment needs, read in one go (the
// stores of one placement would otherwise make the compiler read the next
// segment's values again, each after a wait)
struct PlaceSeg {
    int64_t base;                 // first slot
    unsigned long long *S;        // the species' deposit row of the instance
    uint32_t cap, count;          // slots, occupied slots before this step's creations
    int inst;
};

__device__ __forceinline__ PlaceSeg place_seg(const Dev &d, int seg)
{
    const SegConst &sc = d.segc[seg];
    return PlaceSeg{sc.base, d.S + sc.sp * d.G + sc.gnode, sc.cap, d.segd[seg].count, sc.inst};
}

// write one created particle into segment ps at in-segment index i
// (ignored, and flagged, when the segment is full)
__device__ __forceinline__ void place(const Dev &d, int cur, bool f64, const PlaceSeg &ps, int64_t i,
                                      unsigned long long id, int32_t cell, float f, double x,
                                      double vx, double vy, double vz)
{
    if (i >= (int64_t)ps.cap) {
        atomicOr(&d.instd[ps.inst].status, PIC_ST_CAPACITY);
        return;
    }
    const int64_t g = ps.base + i;
    unsigned long long *S = ps.S;
    int j;
    unsigned long long w1;
    if (f64) {
        ((double *)d.x[cur])[g] = x;
        const double jn = floor(x);
        j = (int)jn;
        w1 = (unsigned long long)rint(ldexp(x - jn, PIC_FRAC_BITS));
    } else {
        ((float *)d.x[cur])[g] = f;
        d.cell[cur][g] = cell;
        j = cell;
        w1 = (unsigned long long)rintf(f * 4294967296.0f);
    }
    st_v(d.vx[cur], g, vx, f64);
    st_v(d.vy[cur], g, vy, f64);
    st_v(d.vz[cur], g, vz, f64);
    store_id(d, cur, g, id);
    if ((1ull << PIC_FRAC_BITS) - w1) atomicAdd(S + j, (1ull << PIC_FRAC_BITS) - w1);
    if (w1) atomicAdd(S + j + 1, w1);
}

// Rank of every ionisation event among the events of its instance, ordered
// by parent id: ev_rank[e] = #{k : inst_k == inst_e, pid_k < pid_e}, and,
// with kinetic neutrals, among those of its cell too (ev_crank).  The pairs
// (event block of kBlock, comparison block of kRankJ) are spread over the
// grid; each adds its partial counts to ev_rank / ev_crank (zero at entry).
__global__ __launch_bounds__(kBlock) void rank_kernel(Dev d)
{
    __shared__ EventIndex X;
    get_event_index(X, d);
    const uint64_t m = X.total;
    const uint64_t ni = (m + kBlock - 1) / kBlock;
    const uint64_t nj = (m + kRankJ - 1) / kRankJ;
    __shared__ unsigned long long s_pid[kRankJ];
    __shared__ int s_inst[kRankJ];
    __shared__ int s_cell[kRankJ];
    const bool cells = d.kinetic_any != 0;
    for (uint64_t p = blockIdx.x; p < ni * nj; p += gridDim.x) {
        const uint64_t bi = p / nj, bj = p - bi * nj;
        // this thread's own event, read before the barrier (beside the
        // column events' reads)
        const uint64_t e = bi * kBlock + threadIdx.x;
        unsigned long long pid = 0;
        int inst = -1, cell = -1;
        if (e < m) {
            const IzEvent &ev = event_at(X, d, (uint32_t)e);
            pid = ev.parent_id;
            inst = ev.inst;
            cell = ev.cell;
        }
        __syncthreads();
        if (threadIdx.x < kRankJ) {
            const uint64_t k = bj * kRankJ + threadIdx.x;
            unsigned long long pid = ~0ull;
            int inst = -2, cell = -1;
            if (k < m) {
                const IzEvent &o = event_at(X, d, (uint32_t)k);
                pid = o.parent_id;
                inst = o.inst;
                cell = o.cell;
            }
            s_pid[threadIdx.x] = pid;
            s_inst[threadIdx.x] = inst;
            s_cell[threadIdx.x] = cell;
        }
        __syncthreads();
        if (e < m) {
            uint32_t r = 0;
#pragma unroll 16
            for (int q = 0; q < kRankJ; ++q) r += (s_inst[q] == inst && s_pid[q] < pid) ? 1u : 0u;
            if (r) atomicAdd(&d.ev_rank[e], r);
            if (cells) {
                uint32_t rc = 0;
                for (int q = 0; q < kRankJ; ++q)
                    rc += (s_inst[q] == inst && s_cell[q] == cell && s_pid[q] < pid) ? 1u : 0u;
                if (rc) atomicAdd(&d.ev_crank[e], rc);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The same ranks for a batch of instances, where events of different
// instances are never compared: the events are counted per instance, the
// counts scanned, each event's (parent id, cell, index) placed in its
// instance's bucket, and every event ranked against its own bucket only
// (sum of m_i^2 comparisons instead of m^2).  Launched when n_inst > 1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void bucket_count_kernel(Dev d)
{
    if ((uint64_t)blockIdx.x * kBlock >= d.glob->ev_total) return;
    __shared__ EventIndex X;
    load_event_index(X, d);
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < X.total; e += gridDim.x * kBlock)
        atomicAdd(&d.inst_ev[event_at(X, d, e).inst], 1u);
}

// one block: inst_start = exclusive prefix of the per-instance counts (which
// are cleared for the next step, as are the fill counters)
__global__ __launch_bounds__(kBlock) void bucket_scan_kernel(Dev d)
{
    __shared__ uint32_t s_w[kWaves];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0u;
    __syncthreads();
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    for (int base = 0; base < d.n_inst; base += kBlock) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < d.n_inst ? d.inst_ev[i] : 0u;
        uint32_t inc = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (lane == 63) s_w[wave] = inc;
        __syncthreads();
        uint32_t run = s_carry + inc - v;
        for (int w = 0; w < wave; ++w) run += s_w[w];
        if (i < d.n_inst) {
            d.inst_start[i] = run;
            d.inst_ev[i] = 0u;
            d.inst_fill[i] = 0u;
        }
        __syncthreads();
        if (threadIdx.x == kBlock - 1) s_carry = run + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) d.inst_start[d.n_inst] = s_carry;
}

__global__ __launch_bounds__(kBlock) void bucket_fill_kernel(Dev d)
{
    if ((uint64_t)blockIdx.x * kBlock >= d.glob->ev_total) return;
    __shared__ EventIndex X;
    load_event_index(X, d);
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < X.total; e += gridDim.x * kBlock) {
        const IzEvent &ev = event_at(X, d, e);
        const uint32_t q = d.inst_start[ev.inst] + atomicAdd(&d.inst_fill[ev.inst], 1u);
        RankEntry r;
        r.pid = ev.parent_id;
        r.cell = ev.cell;
        r.e = e;
        d.rank_bucket[q] = r;
    }
}

// every event against the entries of its instance's bucket
__global__ __launch_bounds__(kBlock) void bucket_rank_kernel(Dev d)
{
    if ((uint64_t)blockIdx.x * kBlock >= d.glob->ev_total) return;
    const uint32_t m = d.glob->ev_total;
    const bool cells = d.kinetic_any != 0;
    // the bucket starts in LDS for the search below (up to kStartLds instances)
    constexpr int kStartLds = 1024;
    __shared__ uint32_t s_start[kStartLds + 1];
    const bool lds = d.n_inst <= kStartLds;
    if (lds)
        for (int i = threadIdx.x; i <= d.n_inst; i += kBlock) s_start[i] = d.inst_start[i];
    __syncthreads();
    const uint32_t *start = lds ? s_start : d.inst_start;
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < m; q += gridDim.x * kBlock) {
        const RankEntry me = d.rank_bucket[q];
        // the instance owning bucket entry q
        int lo = 0, hi = d.n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (start[mid] <= q) lo = mid; else hi = mid - 1;
        }
        const uint32_t b0 = start[lo], b1 = start[lo + 1];
        uint32_t r = 0, rc = 0;
        // (unrolled: eight independent reads of the bucket per wait)
#pragma unroll 8
        for (uint32_t k = b0; k < b1; ++k) {
            const RankEntry o = d.rank_bucket[k];
            const bool less = o.pid < me.pid;
            r += less ? 1u : 0u;
            rc += (less && o.cell == me.cell) ? 1u : 0u;
        }
        d.ev_rank[me.e] = r;
        if (cells) d.ev_crank[me.e] = rc;
    }
}

// ---------------------------------------------------------------------------
// Kinetic neutrals: the atom each ionisation event consumes.  Event e of
// instance i in cell j, with rank q among the events of (i, j), takes the
// (q+1)-th smallest (key, id) among the live atoms in cell j, where key is
// (w0 << 32 | w1) of the atom's Philox block (id, step, 3).  One wave per
// event.  The atoms of cell j are looked up through the cell offsets of the
// last sort over the cells within reach of j: an atom's velocity does not
// change between sorts, so none has moved farther than vmax (steps since the
// sort + nstep) cells.  With no sort yet, or a reach of half the grid, the
// whole species is searched.
// ---------------------------------------------------------------------------
struct KeyId {
    unsigned long long key, id;
    long long slot;
};

__device__ __forceinline__ bool key_less(const KeyId &a, const KeyId &b)
{
    return a.key < b.key || (a.key == b.key && a.id < b.id);
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int o)
{
    const uint32_t lo = __shfl_xor((uint32_t)v, o, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ KeyId wave_min_key(KeyId v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        KeyId w;
        w.key = shfl_xor_u64(v.key, o);
        w.id = shfl_xor_u64(v.id, o);
        w.slot = (long long)shfl_xor_u64((unsigned long long)v.slot, o);
        if (key_less(w, v)) v = w;
    }
    return v;
}

__global__ __launch_bounds__(kBlock) void target_kernel(Dev d)
{
    __shared__ EventIndex X;
    get_event_index(X, d);
    if ((uint64_t)blockIdx.x * kWaves >= X.total) return;  // no event for this block
    const int cur = d.glob->cur_set;
    const bool f64 = (d.precision == PIC_FP64);
    const uint32_t since = d.glob->since_sort;
    const int lane = lane_id();
    const uint32_t n_waves = gridDim.x * kWaves;
    for (uint32_t e = blockIdx.x * kWaves + (threadIdx.x >> 6); e < X.total; e += n_waves) {
        const IzEvent &ev = event_at(X, d, e);
        const InstConst &ic = d.instc[ev.inst];
        long long target = -1;
        if (ic.seg_n >= 0) {
            const SegConst &sn = d.segc[ic.seg_n];
            const long long step = d.instd[ev.inst].step;
            const int64_t nc = ic.nc;
            const int64_t j = ev.cell;
            const uint32_t q = d.ev_crank[e];
            // in-segment slot ranges [a0, b0) and [a1, b1) to search
            int64_t a0 = 0, b0 = d.segd[ic.seg_n].count, a1 = 0, b1 = 0;
            if (since != kNoIndex) {
                const double vmax = __longlong_as_double((long long)d.segd[ic.seg_n].vmax_bits);
                const double reach = vmax * ((double)since + sn.ms);
                if (reach < 0.25 * (double)nc) {
                    const int64_t W = (int64_t)floor(reach) + 1;
                    const uint32_t *off = d.offsets + (int64_t)sn.sp * d.G + sn.gnode;
                    int64_t lo = j - W, hi = j + W;  // cells, inclusive
                    if (ic.bc == PIC_BC_PERIODIC) {
                        if (lo < 0) {
                            a0 = off[lo + nc]; b0 = off[nc]; a1 = 0; b1 = off[hi + 1];
                        } else if (hi >= nc) {
                            a0 = off[lo]; b0 = off[nc]; a1 = 0; b1 = off[hi + 1 - nc];
                        } else {
                            a0 = off[lo]; b0 = off[hi + 1];
                        }
                    } else {
                        lo = lo < 0 ? 0 : lo;
                        hi = hi > nc - 1 ? nc - 1 : hi;
                        a0 = off[lo]; b0 = off[hi + 1];
                    }
                }
            }
            KeyId prev = {0ull, 0ull, -1};
            for (uint32_t r = 0; r <= q; ++r) {
                KeyId best = {~0ull, ~0ull, -1};
                for (int part = 0; part < 2; ++part) {
                    const int64_t a = part ? a1 : a0, b = part ? b1 : b0;
                    for (int64_t i = a + lane; i < b; i += 64) {
                        const int64_t g = sn.base + i;
                        int64_t cj;
                        if (f64) {
                            const double x = ((const double *)d.x[cur])[g];
                            cj = x >= 0.0 ? (int64_t)x : -1;
                        } else {
                            cj = d.cell[cur][g];
                        }
                        if (cj != j) continue;
                        const unsigned long long id = load_id(d, cur, g);
                        const uint4 u = draw(id, step, 3, sn.key0, sn.key1);
                        const KeyId k = {((unsigned long long)u.x << 32) | u.y, id, (long long)g};
                        if ((r == 0 || key_less(prev, k)) && key_less(k, best)) best = k;
                    }
                }
                best = wave_min_key(best);
                if (best.slot < 0) {
                    target = -1;
                    break;
                }
                prev = best;
                target = best.slot;
            }
        }
        if (lane == 0) d.ev_target[e] = target;
    }
}

// the consumed atom at slot t leaves its segment: marked absorbed, its share
// of the deposit taken back (it was deposited by this step's push)
__device__ __forceinline__ void consume_atom(const Dev &d, int cur, bool f64, int seg_n, int64_t t)
{
    const SegConst &sn = d.segc[seg_n];
    unsigned long long *S = d.S + (int64_t)sn.sp * d.G + sn.gnode;
    int j;
    unsigned long long w1;
    if (f64) {
        double *X = (double *)d.x[cur];
        const double x = X[t];
        const double jn = floor(x);
        j = (int)jn;
        w1 = (unsigned long long)rint(ldexp(x - jn, PIC_FRAC_BITS));
        X[t] = kDeadX;
    } else {
        const float f = ((const float *)d.x[cur])[t];
        j = d.cell[cur][t];
        w1 = (unsigned long long)rintf(f * 4294967296.0f);
        d.cell[cur][t] = kDeadCell;
    }
    const unsigned long long w0 = (1ull << PIC_FRAC_BITS) - w1;
    if (w0) atomicAdd(S + j, 0ull - w0);
    if (w1) atomicAdd(S + j + 1, 0ull - w1);
    atomicAdd(&d.segd[seg_n].consumed_step, 1u);
    atomicAdd(&d.instd[sn.inst].n_consumed, 1ull);
}

// the pair of ionisation event e (rank: its rank among its instance's events
// by parent id): the electron at in-segment index count + rank with id
// next_id + 2 rank, the ion after it
__device__ __forceinline__ void emit_ionisation(const Dev &d, int cur, bool f64, uint32_t e, const IzEvent &ev,
                                                uint32_t rank)
{
    const SegConst &se = d.segc[ev.seg];
    const int seg_i = se.partner;
    const SegConst &si = d.segc[seg_i];
    const InstDyn &idn = d.instd[ev.inst];
    const long long step = idn.step;
    const unsigned long long nid = idn.next_id + 2ull * rank;
    // everything the placements read, before their first store
    const PlaceSeg pe = place_seg(d, ev.seg), pi = place_seg(d, seg_i);
    const double sig_n = si.sig_n;
    const int seg_n = d.instc[ev.inst].seg_n;
    // position of the parent (unchanged by the collision)
    int32_t cell = 0;
    float f = 0.f;
    double x = 0.0;
    if (f64) x = ((const double *)d.x[cur])[ev.slot];
    else {
        cell = d.cell[cur][ev.slot];
        f = ((const float *)d.x[cur])[ev.slot];
    }
    const uint4 u1 = draw(ev.parent_id, step, 1, se.key0, se.key1);
    const uint4 u2 = draw(ev.parent_id, step, 2, se.key0, se.key1);
    double d0, d1, d2;
    iso_dir(u1.z, u1.w, d0, d1, d2);
    double n0, n1, n2, n3;
    box_muller(u2.x, u2.y, n0, n1);
    box_muller(u2.z, u2.w, n2, n3);
    place(d, cur, f64, pe, (int64_t)pe.count + rank, nid, cell, f, x,
          ev.g2 * d0, ev.g2 * d1, ev.g2 * d2);
    // the ion: Maxwellian at the parent, or the consumed atom itself
    double ivx = sig_n * n0, ivy = sig_n * n1, ivz = sig_n * n2;
    if (seg_n >= 0) {
        const long long t = d.ev_target[e];
        if (t >= 0) {
            if (f64) {
                x = ((const double *)d.x[cur])[t];
                ivx = ((const double *)d.vx[cur])[t];
                ivy = ((const double *)d.vy[cur])[t];
                ivz = ((const double *)d.vz[cur])[t];
            } else {
                cell = d.cell[cur][t];
                f = ((const float *)d.x[cur])[t];
                ivx = (double)((const float *)d.vx[cur])[t];
                ivy = (double)((const float *)d.vy[cur])[t];
                ivz = (double)((const float *)d.vz[cur])[t];
            }
            consume_atom(d, cur, f64, seg_n, t);
        } else {
            atomicAdd(&d.instd[ev.inst].n_iz_untargeted, 1ull);
        }
    }
    place(d, cur, f64, pi, (int64_t)pi.count + rank, nid + 1ull, cell, f, x, ivx, ivy, ivz);
}

// source pair k of instance i (m_i: the instance's ionisation events this
// step, whose pairs take the ids and slots before the source pairs')
__device__ __forceinline__ void emit_source_pair(const Dev &d, int cur, bool f64, int i, uint32_t k, uint32_t m_i)
{
    const InstConst &ic = d.instc[i];
    const InstDyn &idn = d.instd[i];
    const SegConst &se = d.segc[ic.seg_e];
    const SegConst &si = d.segc[ic.seg_i];
    const long long step = idn.step;
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
    // everything the placements read, before their first store
    const PlaceSeg pe = place_seg(d, ic.seg_e), pi = place_seg(d, ic.seg_i);
    const double se_src = se.sig_src, si_src = si.sig_src;
    place(d, cur, f64, pe, (int64_t)pe.count + m_i + k, nid, cell, f, x, se_src * e0, se_src * e1,
          se_src * e2);
    place(d, cur, f64, pi, (int64_t)pi.count + m_i + k, nid + 1ull, cell, f, x, si_src * i0,
          si_src * i1, si_src * i2);
}

// the source pairs of every instance (all threads of every block; barriers
// inside): instance i creates as many pairs as ions it lost this step, from
// the last blocks down, so that they run beside the ionisation pairs (from
// the first blocks up), not after them.  MAXI: instances held in LDS.
template <int MAXI>
__device__ void emit_sources(const Dev &d, const EventIndex &X, int cur, bool f64)
{
    __shared__ uint32_t s_pre[MAXI + 1];
    __shared__ uint32_t s_m[MAXI];
    const uint32_t stride = gridDim.x * kBlock;
    const int n_inst = d.n_inst < MAXI ? d.n_inst : MAXI;
    __syncthreads();
    count_events(X, d, s_m, n_inst);
    {
        // s_pre = exclusive prefix of the instances' source pairs (block scan)
        __shared__ uint32_t s_w[kWaves];
        __shared__ uint32_t s_carry;
        if (threadIdx.x == 0) s_carry = 0u;
        __syncthreads();
        const int lane = lane_id(), wave = threadIdx.x >> 6;
        for (int base = 0; base < n_inst; base += kBlock) {
            const int i = base + threadIdx.x;
            const uint32_t v = i < n_inst ? source_pairs(d, i) : 0u;
            uint32_t inc = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(inc, o, 64);
                if (lane >= o) inc += t;
            }
            if (lane == 63) s_w[wave] = inc;
            __syncthreads();
            uint32_t run = s_carry + inc - v;
            for (int w = 0; w < wave; ++w) run += s_w[w];
            if (i < n_inst) s_pre[i] = run;
            __syncthreads();
            if (threadIdx.x == kBlock - 1) s_carry = run + v;
            __syncthreads();
        }
        if (threadIdx.x == 0) s_pre[n_inst] = s_carry;
        __syncthreads();
    }
    const uint32_t n_src_all = s_pre[n_inst];
    // source pairs from the last blocks down, so that they run beside the
    // ionisation pairs (from the first blocks up), not after them
    const uint32_t sb = gridDim.x - 1 - blockIdx.x;
    for (uint32_t q = sb * kBlock + threadIdx.x; q < n_src_all; q += stride) {
        int lo = 0, hi = n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pre[mid] <= q) lo = mid; else hi = mid - 1;
        }
        emit_source_pair(d, cur, f64, lo, q - s_pre[lo], s_m[lo]);
    }
}

__global__ __launch_bounds__(kBlock) void emit_kernel(Dev d)
{
    __shared__ EventIndex X;
    get_event_index(X, d);
    const int cur = d.glob->cur_set;
    const bool f64 = (d.precision == PIC_FP64);
    const uint32_t m_all = X.total;
    const uint32_t stride = gridDim.x * kBlock;
    // ionisation pairs, ranked by the rank kernels
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < m_all; e += stride)
        emit_ionisation(d, cur, f64, e, event_at(X, d, e), d.ev_rank[e]);
    emit_sources<kMaxInstLds>(d, X, cur, f64);
}

// A single instance without kinetic neutrals: the rank of each ionisation
// event among the step's events by parent id taken here, so that no rank
// kernel runs.  Block b takes the events of group g = b (+ k grid) of 64.
// Every block stages all parent ids in LDS (their loads issued beside the
// group's event loads, once when they fit and every id is below 2^32, else
// per chunk), wave 0 draws everything its 64 pairs need except the rank while
// the other waves compare the group's 64 parent ids (one per lane) against a
// third of the staged ids each, the partial ranks are summed in LDS and wave
// 0 places the 64 pairs.  The constants of the instance's segments are read
// into LDS while the event index is built.
constexpr int kRankChunk = 4096;  // parent ids per LDS chunk

// the constants a pair of a parent segment needs (no kinetic neutrals)
struct PairSeg {
    PlaceSeg pe, pi;  // the electron's and the ion's segment
    uint32_t key0, key1;
    double sig_n;     // the ion segment's neutral Maxwellian
    long long step;
    unsigned long long next_id;
};

// what placing an ionisation pair needs besides its rank
struct IzPair {
    PlaceSeg pe, pi;
    unsigned long long next_id;
    int32_t cell;
    float f;
    double x;
    double ev[3], iv[3];  // velocities of the new electron and ion
};

// the parent's position (unchanged by the collision)
__device__ __forceinline__ void parent_position(const Dev &d, int cur, bool f64, const IzEvent &ev, IzPair &q)
{
    q.cell = 0;
    q.f = 0.f;
    q.x = 0.0;
    if (f64) q.x = ((const double *)d.x[cur])[ev.slot];
    else {
        q.cell = d.cell[cur][ev.slot];
        q.f = ((const float *)d.x[cur])[ev.slot];
    }
}

// the draws and velocities of event ev's pair, with its segment's constants
__device__ __forceinline__ void prepare_pair(const PairSeg &P, const IzEvent &ev, IzPair &q)
{
    q.next_id = P.next_id;
    q.pe = P.pe;
    q.pi = P.pi;
    const uint4 u1 = draw(ev.parent_id, P.step, 1, P.key0, P.key1);
    const uint4 u2 = draw(ev.parent_id, P.step, 2, P.key0, P.key1);
    double d0, d1, d2;
    iso_dir(u1.z, u1.w, d0, d1, d2);
    double n0, n1, n2, n3;
    box_muller(u2.x, u2.y, n0, n1);
    box_muller(u2.z, u2.w, n2, n3);
    q.ev[0] = ev.g2 * d0;
    q.ev[1] = ev.g2 * d1;
    q.ev[2] = ev.g2 * d2;
    q.iv[0] = P.sig_n * n0;
    q.iv[1] = P.sig_n * n1;
    q.iv[2] = P.sig_n * n2;
}

// every parent id of the step into LDS, by region rather than by event:
// thread t takes regions t, t + kBlock, ... and loads up to kStageK events of
// each of its first kStageRows regions before its first wait (a region rarely
// holds more; the rest, further regions and the overflow list follow in
// plain loops).  The first regions' loads and stores are separate calls, so
// that a block can issue other loads between them; staging all of a thread's
// regions at once would hold twice the registers and halve the kernel's
// waves per SIMD.  T: the id (unsigned long long) or its low word (uint32_t,
// when every id is below 2^32).
constexpr int kStageK = 4;
constexpr int kStageRows = 4;  // regions per thread staged at once (all of them up to 1024 regions)

template <typename T>
__device__ __forceinline__ T pid_of(const IzEvent &ev)
{
    if constexpr (sizeof(T) == 4) return *reinterpret_cast<const uint32_t *>(&ev.parent_id);  // the low word
    else return ev.parent_id;
}

template <typename T>
struct PidStage {
    T v[kStageRows][kStageK];
    uint32_t dst[kStageRows], n[kStageRows];
};

// the regions threadIdx.x + (r0 + r) kBlock, r < kStageRows
template <typename T>
__device__ __forceinline__ void stage_pids_load(const EventIndex &X, const Dev &d, int r0, PidStage<T> &P)
{
    const int nb = d.n_push_blocks;
#pragma unroll
    for (int r = 0; r < kStageRows; ++r) {
        const int b = threadIdx.x + (r0 + r) * kBlock;
        const bool ok = b < nb;
        P.dst[r] = ok ? X.pre[b] : 0u;
        P.n[r] = ok ? X.pre[b + 1] - X.pre[b] : 0u;
#pragma unroll
        for (int k = 0; k < kStageK; ++k)
            P.v[r][k] = ((uint32_t)k < P.n[r]) ? pid_of<T>(d.ev[(int64_t)b * d.ev_q + k]) : T(0);
    }
}

template <typename T>
__device__ __forceinline__ void stage_pids_put(const Dev &d, int r0, const PidStage<T> &P, T *s)
{
#pragma unroll
    for (int r = 0; r < kStageRows; ++r) {
#pragma unroll
        for (int k = 0; k < kStageK; ++k)
            if ((uint32_t)k < P.n[r]) s[P.dst[r] + k] = P.v[r][k];
        const int b = threadIdx.x + (r0 + r) * kBlock;
        for (uint32_t k = kStageK; k < P.n[r]; ++k) s[P.dst[r] + k] = pid_of<T>(d.ev[(int64_t)b * d.ev_q + k]);
    }
}

// the rest after the first kStageRows rows: the other regions, and the
// overflow list
template <typename T>
__device__ __forceinline__ void stage_pids_rest(const EventIndex &X, const Dev &d, T *s)
{
    for (int r0 = kStageRows; r0 * kBlock < d.n_push_blocks; r0 += kStageRows) {  // uniform
        PidStage<T> P;
        stage_pids_load<T>(X, d, r0, P);
        stage_pids_put<T>(d, r0, P, s);
    }
    for (uint32_t e = X.in_regions + threadIdx.x; e < X.total; e += kBlock)
        s[e] = pid_of<T>(d.ev[(int64_t)d.n_regions * d.ev_q + (e - X.in_regions)]);
}

__global__ __launch_bounds__(kBlock) void emit_ranked_kernel(Dev d)
{
    __shared__ EventIndex X;
    __shared__ __align__(16) unsigned long long s_pid[kRankChunk];
    __shared__ uint32_t s_part[kWaves][64];
    __shared__ PairSeg s_ps[PIC_MAX_SPECIES];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t n_src = source_pairs(d, 0);  // read first: in flight beside the index
    // the constants of the instance's segments (one thread each; per-lane
    // loads, which unlike uniform scalar loads do not hold up the index's
    // LDS operations), into LDS once the index is built
    const int nsp = d.n_seg;  // a single instance: its segments are 0 .. nsp - 1
    PairSeg ps = {};
    const bool ps_mine = wave == 0 && lane < nsp && d.segc[lane].partner >= 0;
    build_event_index(X, d);
    if (ps_mine) {
        const SegConst &se = d.segc[lane];
        const InstDyn &idn = d.instd[se.inst];
        ps.pe = place_seg(d, lane);
        ps.pi = place_seg(d, se.partner);
        ps.key0 = se.key0;
        ps.key1 = se.key1;
        ps.sig_n = d.segc[se.partner].sig_n;
        ps.step = idn.step;
        ps.next_id = idn.next_id;
    }
    const int cur = d.glob->cur_set;
    const bool f64 = (d.precision == PIC_FP64);
    const uint32_t m = X.total;
    const uint32_t n_groups = (m + 63u) / 64u;
    if (blockIdx.x == 0 && threadIdx.x == 0) d.glob->ev_total = m;  // for the close kernel
    // every id below 2^32: the ranks compare the low words, four per LDS read
    const bool narrow = d.instd[0].wide_ids == 0u && m <= (uint32_t)kRankChunk;
    uint32_t *s_pid32 = reinterpret_cast<uint32_t *>(s_pid);
    bool staged = false;  // the narrow ids are in LDS (block-uniform)
    for (uint32_t g = blockIdx.x; g < n_groups; g += gridDim.x) {  // block-uniform
        const uint32_t e = g * 64u + (uint32_t)lane;
        const bool mine = e < m;
        PidStage<uint32_t> P32;
        if (narrow && !staged) stage_pids_load<uint32_t>(X, d, 0, P32);
        IzEvent ev = {};
        if (mine) ev = event_at(X, d, e);
        IzPair q = {};
        if (wave == 0 && mine) parent_position(d, cur, f64, ev, q);
        if (ps_mine) s_ps[lane] = ps;
        uint32_t r = 0;
        if (narrow) {
            if (!staged) {
                stage_pids_put<uint32_t>(d, 0, P32, s_pid32);
                stage_pids_rest<uint32_t>(X, d, s_pid32);
                const uint32_t n4 = (m + 3u) & ~3u;  // padded with ids no parent has below it
                for (uint32_t i = m + threadIdx.x; i < n4; i += kBlock) s_pid32[i] = 0xFFFFFFFFu;
                staged = true;
            }
            __syncthreads();
            if (wave == 0 && mine) prepare_pair(s_ps[ev.seg], ev, q);
            // waves 1 .. kWaves - 1 compare while wave 0 draws
            const uint32_t n4 = (m + 3u) & ~3u;
            const uint32_t wc = wave > 0 ? (uint32_t)wave - 1u : 0u;
            const uint32_t q0 = (wc * (n4 / 4u) / (kWaves - 1)) * 4u;
            const uint32_t q1 = ((wc + 1u) * (n4 / 4u) / (kWaves - 1)) * 4u;
            if (mine && wave > 0) {
                const uint32_t pid = (uint32_t)ev.parent_id;
#pragma unroll 4
                for (uint32_t k = q0; k < q1; k += 4) {
                    const uint4 v = *reinterpret_cast<const uint4 *>(&s_pid32[k]);
                    r += (v.x < pid ? 1u : 0u) + (v.y < pid ? 1u : 0u) + (v.z < pid ? 1u : 0u) +
                         (v.w < pid ? 1u : 0u);
                }
            }
        } else {
            for (uint32_t c0 = 0; c0 < m; c0 += kRankChunk) {
                const uint32_t cn = min((uint32_t)kRankChunk, m - c0);
                __syncthreads();  // the previous chunk's readers are done (and s_ps is in place)
                if (c0 == 0 && wave == 0 && mine) prepare_pair(s_ps[ev.seg], ev, q);
                if (m <= (uint32_t)kRankChunk) {
                    PidStage<unsigned long long> P64;
                    stage_pids_load<unsigned long long>(X, d, 0, P64);
                    stage_pids_put<unsigned long long>(d, 0, P64, s_pid);
                    stage_pids_rest<unsigned long long>(X, d, s_pid);
                } else {
                    for (uint32_t i = threadIdx.x; i < cn; i += kBlock) s_pid[i] = event_at(X, d, c0 + i).parent_id;
                }
                __syncthreads();
                // the first chunk: waves 1 .. kWaves - 1 compare while wave 0 draws
                const uint32_t nw = c0 == 0 ? (uint32_t)kWaves - 1u : (uint32_t)kWaves;
                const uint32_t wc = c0 == 0 ? (wave > 0 ? (uint32_t)wave - 1u : 0u) : (uint32_t)wave;
                const uint32_t q0 = wc * cn / nw, q1 = (wc + 1u) * cn / nw;
                if (mine && (c0 > 0 || wave > 0)) {
                    const unsigned long long pid = ev.parent_id;
#pragma unroll 8
                    for (uint32_t k = q0; k < q1; ++k) r += s_pid[k] < pid ? 1u : 0u;
                }
            }
        }
        s_part[wave][lane] = r;
        __syncthreads();
        if (wave == 0 && mine) {
            uint32_t rank = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) rank += s_part[w][lane];
            const unsigned long long nid = q.next_id + 2ull * rank;
            place(d, cur, f64, q.pe, (int64_t)q.pe.count + rank, nid, q.cell, q.f, q.x, q.ev[0], q.ev[1], q.ev[2]);
            place(d, cur, f64, q.pi, (int64_t)q.pi.count + rank, nid + 1ull, q.cell, q.f, q.x, q.iv[0], q.iv[1],
                  q.iv[2]);
        }
        __syncthreads();  // s_part is free for the next group
    }
    // the source pairs, from the last blocks down
    const uint32_t sb = gridDim.x - 1 - blockIdx.x;
    for (uint32_t k = sb * kBlock + threadIdx.x; k < n_src; k += gridDim.x * kBlock)
        emit_source_pair(d, cur, f64, 0, k, m);
}

__global__ __launch_bounds__(kBlock) void close_step_kernel(Dev d, int with_events)
{
    close_step(d, with_events);
}

hipError_t launch_collide(const Dev &d, hipStream_t st, bool overflow_only)
{
    const size_t lds = d.n_seg <= kCntSegMax ? sizeof(uint32_t) * d.n_seg * kNCnt : 0;
    if (overflow_only) {
        const dim3 grid(kOvfCollideBlocks);
        if (d.n_seg <= kCollSegLds)
            hipLaunchKernelGGL((collide_kernel<true, true>), grid, dim3(kBlock), lds, st, d);
        else
            hipLaunchKernelGGL((collide_kernel<false, true>), grid, dim3(kBlock), lds, st, d);
    } else if (d.n_seg <= kCollSegLds) {
        hipLaunchKernelGGL((collide_kernel<true, false>), dim3(d.n_push_blocks), dim3(kBlock), lds, st, d);
    } else {
        hipLaunchKernelGGL((collide_kernel<false, false>), dim3(d.n_push_blocks), dim3(kBlock), lds, st, d);
    }
    return hipGetLastError();
}

hipError_t launch_emit(const Dev &d, hipStream_t st, bool pairs, bool events, int *deferred_close)
{
    auto close = [&](int mode) {
        if (deferred_close) {
            *deferred_close = mode;
            return hipSuccess;
        }
        hipLaunchKernelGGL(close_step_kernel, dim3(1), dim3(kBlock), 0, st, d, mode);
        return hipGetLastError();
    };
    if (events && d.n_inst > 1) {  // a single instance builds the index in each kernel
        hipLaunchKernelGGL(index_kernel, dim3(1), dim3(kBlock), 0, st, d);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (events && d.n_inst == 1 && !d.kinetic_any && pairs) {
        // ranks inside the emit kernel
        hipLaunchKernelGGL(emit_ranked_kernel, dim3(kEmitRankedBlocks), dim3(kBlock), 0, st, d);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return close(2);
    }
    if (events) {
        hipError_t e;
        if (d.n_inst > 1) {
            hipLaunchKernelGGL(bucket_count_kernel, dim3(kRankBlocks), dim3(kBlock), 0, st, d);
            hipLaunchKernelGGL(bucket_scan_kernel, dim3(1), dim3(kBlock), 0, st, d);
            hipLaunchKernelGGL(bucket_fill_kernel, dim3(kRankBlocks), dim3(kBlock), 0, st, d);
            hipLaunchKernelGGL(bucket_rank_kernel, dim3(kRankBlocks), dim3(kBlock), 0, st, d);
        } else {
            hipLaunchKernelGGL(rank_kernel, dim3(kRankBlocks), dim3(kBlock), 0, st, d);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (d.kinetic_any) {
            hipLaunchKernelGGL(target_kernel, dim3(kTargetBlocks), dim3(kBlock), 0, st, d);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    if (pairs) {
        hipLaunchKernelGGL(emit_kernel, dim3(kEmitBlocks), dim3(kBlock), 0, st, d);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return close(events ? 1 : 0);
}

}  // namespace picx
