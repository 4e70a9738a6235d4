// push.hip -- the mover (paper Sec. 2, phase 5; moveb listing of Sec. 6) and
// the fixed-point charge deposition (Sec. 2, phase 1) for gfx950.
//
// One pass per particle and step: linear gather of the grid acceleration at
// the in-cell offset, magnetised Boris velocity update, advance
// x += nstep vx (a subcycled species moves every nstep steps over nstep dt
// and is only deposited in between),
// absorbing or periodic walls, the null-collision candidate test (one Philox
// block keyed by id and step), and the deposit of the new position.
//
// Memory plan (HBM-bound):
//  * structure-of-arrays streamed once, with nontemporal loads and stores;
//    a block owns a tile of kTile consecutive slots of one segment, and every
//    wave issues the loads of all its kPer 64-slot chunks before computing,
//    so each wave keeps kPer x (4 + 4 + 12 + 8) bytes x 64 lanes in flight;
//  * tile base pointers live in scalar registers; lanes address them with a
//    32-bit offset below kTile;
//  * segment tables and counts are staged in LDS once per launch, so no
//    global load sits on the critical path between tiles;
//  * the deposit of cell-sorted neighbours is summed first over runs of equal
//    cells inside each wave, then into the wave's own LDS window of nodes
//    (no block barrier), and the window is flushed with one 64-bit global
//    atomic per touched node per wave and tile;
//  * each candidate, with its velocity after the push and its id, goes to its
//    block's own region of the candidate list (index from an LDS counter), so
//    the collide kernel reads them contiguously; only a block with more than
//    its region's cand_q candidates appends the excess to a shared overflow
//    list.
#include "collide_common.h"
#include "mover_common.h"
#include "tile_queue.h"

#pragma clang fp contract(off)

namespace picx {

constexpr int kSegLds = 1024;     // segments whose tables are staged in LDS

struct PushLds {
    unsigned long long wdep[kWaves][kWaveWin];  // each wave's deposit window
    int64_t tile0[kSegLds + 1];
    int64_t base[kSegLds];
    uint32_t count[kSegLds];
    uint8_t flg[kSegLds];   // kFlgTest | kFlgForce | kFlgWide of each segment
    uint32_t live0[kSegLds + 1];  // the movers: live tiles of the segments before each
};

// per-segment flags of the movers: a collision process (the candidate test
// reads ids and draws), a field that acts (the gather), some id of the
// instance at or above 2^32 (the test reads the ids' high words too; fixed
// for the length of a launch)
constexpr uint32_t kFlgTest = 1u, kFlgForce = 2u, kFlgWide = 4u;

__device__ __forceinline__ uint32_t seg_flags(const Dev &d, int s)
{
    const SegConst &sc = d.segc[s];
    return (sc.T != 0ull ? kFlgTest : 0u) | (sc.force ? kFlgForce : 0u) |
           (d.instd[sc.inst].wide_ids != 0u ? kFlgWide : 0u);
}

// a subcycled species between its pushes (block-uniform)
__device__ __forceinline__ bool still(const Dev &d, int seg)
{
    const SegConst &sc = d.segc[seg];
    return sc.nstep > 1 && d.instd[sc.inst].step % sc.nstep != 0;
}

// drop_still: a subcycled species between its pushes gets no tiles (its
// segments read as empty, so the movers pay nothing per tile for the test)
__device__ __forceinline__ void push_lds_init(PushLds &L, const Dev &d, bool drop_still = false)
{
    for (int i = threadIdx.x; i < kWaves * kWaveWin; i += kBlock) (&L.wdep[0][0])[i] = 0ull;
    if (d.n_seg <= kSegLds) {
        for (int s = threadIdx.x; s <= d.n_seg; s += kBlock) {
            L.tile0[s] = d.seg_tile0[s];
            if (s < d.n_seg) {
                L.base[s] = d.seg_base[s];
                L.count[s] = drop_still && still(d, s) ? 0 : d.segd[s].count;
                L.flg[s] = (uint8_t)seg_flags(d, s);
            }
        }
    }
    __syncthreads();
}

// a block-uniform value moved to scalar registers (the compiler cannot see
// that values read from LDS are the same in every lane)
__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// (segment, first slot, occupied slots, flags) of virtual tile t.  hint:
// the segment of the block's previous tile (tiles only increase), so a few
// steps forward usually find it; otherwise a binary search.
__device__ __forceinline__ int tile_seg(const PushLds &L, const Dev &d, int64_t t, int64_t &tile0,
                                        int64_t &base, int64_t &count, uint32_t &flags, int &hint)
{
    int seg;
    if (d.n_seg <= kSegLds) {
        int s = hint, steps = 0;
        while (s + 1 < d.n_seg && L.tile0[s + 1] <= t && steps < 8) {
            ++s;
            ++steps;
        }
        if (s + 1 < d.n_seg && L.tile0[s + 1] <= t) {
            int lo = s, hi = d.n_seg - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (L.tile0[mid] <= t) lo = mid; else hi = mid - 1;
            }
            s = lo;
        }
        seg = __builtin_amdgcn_readfirstlane(s);
        hint = seg;
        tile0 = L.tile0[seg];
        base = L.base[seg];
        count = L.count[seg];
        flags = L.flg[seg];
    } else {
        seg = seg_of_tile(d.seg_tile0, d.n_seg, t);
        tile0 = d.seg_tile0[seg];
        base = d.seg_base[seg];
        count = d.segd[seg].count;
        flags = seg_flags(d, seg);
    }
    tile0 = uniform_i64(tile0);
    base = uniform_i64(base);
    count = uniform_i64(count);
    flags = (uint32_t)__builtin_amdgcn_readfirstlane((int)flags);
    return __builtin_amdgcn_readfirstlane(seg);
}

// Deposit the kPer chunks of this wave through its own LDS window (no block
// barrier: the waves of a block run through their tiles independently).
template <int NP>
__device__ __forceinline__ void deposit_tile(PushLds &L, unsigned long long *__restrict__ S,
                                             const int (&key)[NP], const unsigned long long (&w1)[NP])
{
    deposit_wave<NP>(L.wdep[threadIdx.x >> 6], S, key, w1);
}

// The deposit of the current positions of one tile (both forms): the
// standalone deposit, and a subcycled species between its pushes.
__device__ __forceinline__ void deposit_positions(PushLds &L, const Dev &d, int cur, const SegConst &sc,
                                                  int64_t tb, uint32_t rem)
{
    unsigned long long *__restrict__ S = d.S + sc.sp * d.G + sc.gnode;
    const bool f64 = (d.precision == PIC_FP64);
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    int key[kPer];
    unsigned long long w1[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const uint32_t o = (uint32_t)((wave * kPer + k) * 64 + lane);
        key[k] = -1;
        w1[k] = 0;
        if (o < rem) {
            if (f64) {
                const double x = stream_ld(&((const double *)d.x[cur])[tb + o]);
                if (x >= 0.0) {
                    const double jn = floor(x);
                    key[k] = (int)jn;
                    w1[k] = (unsigned long long)rint(ldexp(x - jn, PIC_FRAC_BITS));
                }
            } else {
                const int32_t jj = stream_ld(&d.cell[cur][tb + o]);
                if (jj >= 0) {
                    key[k] = jj;
                    w1[k] = (unsigned long long)rintf(stream_ld(&((const float *)d.x[cur])[tb + o]) *
                                                      4294967296.0f);
                }
            }
        }
    }
    deposit_tile<kPer>(L, S, key, w1);
}

// A candidate is written, with its velocity after the push and its id, to
// its wave's own part of the block's region of the candidate list: the
// wave's running count wn is block-uniform per wave (a scalar), so no LDS or
// global atomic is needed; a wave whose part is full appends the excess to
// the shared overflow list.
template <typename V>
__device__ __forceinline__ void queue_candidate(const Dev &d, bool cand, uint32_t g, int seg, int inst,
                                                V vx, V vy, V vz, unsigned long long pid, uint32_t &wn)
{
    const unsigned long long m = ballot(cand);
    if (!m) return;
    const int lane = lane_id();
    const uint32_t n = (uint32_t)__popcll(m);
    const uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    const uint32_t base = wn;
    wn = base + n;
    const uint32_t qw = (uint32_t)d.cand_q / kWaves;
    // the first n_reg candidates fill the rest of the wave's part, the others overflow
    const uint32_t room = base < qw ? qw - base : 0u;
    const uint32_t n_reg = n < room ? n : room;
    uint32_t gb = 0;
    if (n_reg != n) {
        const int leader = __ffsll((long long)m) - 1;
        if (lane == leader) gb = atomicAdd(&d.glob->cand_ovf, n - n_reg);
        gb = __shfl(gb, leader, 64);
    }
    if (!cand) return;
    int64_t idx;
    if (rank < n_reg) {
        idx = (int64_t)blockIdx.x * d.cand_q + (int64_t)(threadIdx.x >> 6) * qw + base + rank;
    } else {
        const uint32_t o = gb + (rank - n_reg);
        if (o >= (uint32_t)d.cand_ovf_cap) {
            atomicOr(&d.instd[inst].status, PIC_ST_CANDIDATES);
            return;
        }
        idx = (int64_t)d.n_regions * d.cand_q + o;
    }
    Cand c;
    c.g = g;
    c.seg = seg;
    c.vx = (double)vx;
    c.vy = (double)vy;
    c.vz = (double)vz;
    c.pid = pid;
    d.cand[idx] = c;
}

// the number of entries in this wave's part of the region
__device__ __forceinline__ void flush_candidates(const Dev &d, uint32_t wn)
{
    const uint32_t qw = (uint32_t)d.cand_q / kWaves;
    if (lane_id() == 0) d.cand_n[blockIdx.x * kWaves + (threadIdx.x >> 6)] = min(wn, qw);
}

// After its push the block collides the candidates of its own region (no
// other block writes or reads it): once every wave has passed the barrier,
// its candidate entries and its particles' new velocities are in place.  The
// process counts take the LDS of the tile tables, which the push no longer
// needs.  Overflowed candidates are left to the collide kernel.
__device__ __forceinline__ void collide_own_region(PushLds &L, const Dev &d, uint32_t wn)
{
    __shared__ uint32_t s_wn[kWaves];
    __shared__ uint32_t s_en;
    __shared__ SegConst s_sc[kCollSegLds];
    __shared__ long long s_step[kCollSegLds];
    const uint32_t qw = (uint32_t)d.cand_q / kWaves;
    if (lane_id() == 0) s_wn[threadIdx.x >> 6] = min(wn, qw);
    __syncthreads();
    constexpr size_t kTables = sizeof(L.tile0) + sizeof(L.base) + sizeof(L.count) + sizeof(L.flg);
    uint32_t *s_cnt = reinterpret_cast<uint32_t *>(&L.tile0[0]);
    const bool lds_cnt = (size_t)d.n_seg * kNCnt * sizeof(uint32_t) <= kTables;
    if (d.n_seg <= kCollSegLds)
        collide_block<true>(d, blockIdx.x, true, false, s_wn, s_cnt, lds_cnt, s_en, s_sc, s_step);
    else
        collide_block<false>(d, blockIdx.x, true, false, s_wn, s_cnt, lds_cnt, s_en, s_sc, s_step);
}

// ---------------------------------------------------------------------------
// FP32 form: (int32 cell, float f in [0,1), float v), FP32 gather and push
// ---------------------------------------------------------------------------
template <bool DEP, bool MCC, int NP, bool COLL>
__global__ __launch_bounds__(kBlock) void push_f32_kernel(Dev d)
{
    __shared__ PushLds L;
    push_lds_init(L, d, true);
    const int cur = d.glob->cur_set;
    float *__restrict__ X = (float *)d.x[cur];
    int32_t *__restrict__ CELL = d.cell[cur];
    float *__restrict__ VX = (float *)d.vx[cur];
    float *__restrict__ VY = (float *)d.vy[cur];
    float *__restrict__ VZ = (float *)d.vz[cur];
    const uint32_t *__restrict__ IDL = d.id_lo[cur];
    const uint32_t *__restrict__ IDH = d.id_hi[cur];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    uint32_t wn = 0;  // this wave's candidates so far (uniform)
    // the deposit window of the wave's previous pass, flushed once the next
    // pass's loads are issued when d.late_flush (its global atomics would
    // otherwise stand, on the in-order memory counter, between those loads
    // and their wait), else at the end of its own pass
    int dlo = 0, dspan = 0;
    unsigned long long *dS = nullptr;

    int hint = 0;  // segment of the previous tile
    // the constants of the segment of the previous tile, kept across tiles
    // (loaded again only when the segment changes, so no global load of
    // them waits behind a tile's particle loads)
    int cseg = -1;
    const float *__restrict__ acc = nullptr;
    unsigned long long *__restrict__ S = nullptr;
    int nc = 0, inst = 0;
    bool periodic = false;
    float tx = 0.f, ty = 0.f, sx = 0.f, sy = 0.f, msf = 0.f, hk = 0.f;
    uint32_t key0 = 0, key1 = 0;
    unsigned long long T = 0;
    long long step = 0;
    const uint32_t n_live = d.n_seg <= kSegLds ? live_tiles_init<kSegLds>(L, d) : (uint32_t)d.n_tiles;
    TileQueue Q;
    tile_queue_init(Q, d, n_live);
    int lhint = 0;  // segment of the previous live tile
    __shared__ int64_t s_next[2];  // the block's next tile, by parity of its tiles
    int par = 0;
    const int q = wave;  // the wave's part of each tile
    const bool w0 = __builtin_amdgcn_readfirstlane(wave) == 0;
    int64_t t = blockIdx.x < n_live ? live_tile<kSegLds>(L, d, blockIdx.x, lhint) : -1;
    if (t >= 0) do {
        int64_t tile0, base, count;
        uint32_t flg;
        const int seg = tile_seg(L, d, t, tile0, base, count, flg, hint);
        const int64_t t0 = (t - tile0) * (int64_t)kTile;
        // a subcycled species between its pushes keeps its positions (their
        // deposit is a launch of its own, deposit_kernel<true>)
        const bool work = t0 < count && !(d.n_seg > kSegLds && still(d, seg));

        // the tile in kPer / NP passes of NP chunks per wave (NP = kPer: one pass)
#pragma unroll 1
        for (int r0 = 0; work && r0 < kPer; r0 += NP) {
            // a species with no collision process takes no test (no id read, no
            // draw); a species on which no field acts takes no gather
            const bool test = MCC && (flg & kFlgTest);
            const bool force = (flg & kFlgForce) != 0;
            // ---- loads of all chunks
            int32_t j[NP];
            float f[NP], vx[NP], vy[NP], vz[NP];
            unsigned long long pid[NP];
            bool lv[NP];
            // the tile's arrays from scalar base pointers; lanes address them with
            // a 32-bit offset below kTile
            const int64_t tb = base + t0;
            const uint32_t rem = (uint32_t)min(count - t0, (int64_t)kTile);
            float *__restrict__ Xt = X + tb;
            int32_t *__restrict__ CELLt = CELL + tb;
            float *__restrict__ VXt = VX + tb;
            float *__restrict__ VYt = VY + tb;
            float *__restrict__ VZt = VZ + tb;
            const uint32_t *__restrict__ IDLt = IDL + tb;
            const uint32_t *__restrict__ IDHt = IDH + tb;
            if (rem == (uint32_t)kTile) {
                // a full tile: every load unconditional, so none is predicated
                // and the wave issues all of them before its first wait
                if (test && !(flg & kFlgWide)) {
                    // every id below 2^32: the low words are the ids
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                        j[k] = stream_ld(&CELLt[o]);
                        f[k] = stream_ld(&Xt[o]);
                        vx[k] = stream_ld(&VXt[o]);
                        vy[k] = stream_ld(&VYt[o]);
                        vz[k] = stream_ld(&VZt[o]);
                        pid[k] = stream_ld(&IDLt[o]);
                    }
                } else if (test) {
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                        j[k] = stream_ld(&CELLt[o]);
                        f[k] = stream_ld(&Xt[o]);
                        vx[k] = stream_ld(&VXt[o]);
                        vy[k] = stream_ld(&VYt[o]);
                        vz[k] = stream_ld(&VZt[o]);
                        pid[k] = (unsigned long long)stream_ld(&IDLt[o]) |
                                 ((unsigned long long)stream_ld(&IDHt[o]) << 32);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                        j[k] = stream_ld(&CELLt[o]);
                        f[k] = stream_ld(&Xt[o]);
                        vx[k] = stream_ld(&VXt[o]);
                        vy[k] = stream_ld(&VYt[o]);
                        vz[k] = stream_ld(&VZt[o]);
                        pid[k] = 0;
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                    j[k] = kDeadCell;
                    f[k] = vx[k] = vy[k] = vz[k] = 0.f;
                    pid[k] = 0;
                    if (o < rem) {
                        j[k] = stream_ld(&CELLt[o]);
                        f[k] = stream_ld(&Xt[o]);
                        vx[k] = stream_ld(&VXt[o]);
                        vy[k] = stream_ld(&VYt[o]);
                        vz[k] = stream_ld(&VZt[o]);
                        if (test) {
                            pid[k] = stream_ld(&IDLt[o]);
                            if (flg & kFlgWide) pid[k] |= (unsigned long long)stream_ld(&IDHt[o]) << 32;
                        }
                    }
                }
            }
            if (DEP && dspan > 0) {
                deposit_flush(L.wdep[wave], dS, dlo, dspan);
                dspan = 0;
            }
            if (w0 && r0 == 0) tile_grab(Q);  // the next tile, behind this one's loads
#pragma unroll
            for (int k = 0; k < NP; ++k) lv[k] = j[k] >= 0;
            // the segment's constants, read once the tile's loads are issued
            // (their scalar loads share a counter with the LDS reads that
            // address the tile: read first, the tile's loads would wait for them)
            if (r0 == 0 && seg != cseg) {
                const SegConst &sc = d.segc[seg];
                acc = d.acc32 + sc.sp * d.G + sc.gnode;
                S = d.S + sc.sp * d.G + sc.gnode;
                nc = sc.nc;
                periodic = (sc.bc == PIC_BC_PERIODIC);
                tx = sc.txf, ty = sc.tyf, sx = sc.sxf, sy = sc.syf;
                msf = sc.msf, hk = 0.5f * sc.msf;
                key0 = sc.key0, key1 = sc.key1;
                T = sc.T;
                inst = sc.inst;
                if (MCC) step = d.instd[inst].step;
                cseg = seg;
            }
            // ---- gather
            // (unpredicated: an empty slot reads node 0 and ignores it, so the
            // wave issues the four gathers before one wait, not one wait each)
            float a0[NP], a1[NP];
            if (force) {
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const int jj = j[k] >= 0 ? j[k] : 0;
                    a0[k] = acc[jj];
                    a1[k] = acc[jj + 1];
                }
            } else {
#pragma unroll
                for (int k = 0; k < NP; ++k) a0[k] = a1[k] = 0.f;
            }
            // ---- push, walls, candidate test
            // (every lane runs the arithmetic, an empty slot on whatever its
            // registers hold, and only live lanes count or keep a result: so
            // the stored registers are written on every path, and the stores
            // need no wait for the tile's loads, nor for what was issued
            // after them)
            int key[NP];
            unsigned long long w1[NP];
            bool cand[NP];
            bool left = false, right = false, cfl = false, bad = false;
            int n_left = 0, n_right = 0;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                key[k] = -1;
                w1[k] = 0;
                cand[k] = false;
                const bool live = j[k] >= 0;
                const float a = fmaf(f[k], a1[k] - a0[k], a0[k]);
                const float h = hk * a;
                const float mx = vx[k] + h, my = vy[k], mz = vz[k];
                const float px = mx - mz * ty;
                const float py = my + mz * tx;
                const float pz = mz + (mx * ty - my * tx);
                const float qx = mx - pz * sy;
                const float qy = my + pz * sx;
                const float qz = mz + (px * sy - py * sx);
                const float nvx = qx + h, nvy = qy, nvz = qz;
                // advance in cell-relative coordinates; |fl| is clamped so that a
                // runaway (flagged) particle still maps to a valid integer cell
                float fn = f[k] + msf * nvx;
                const float fl = fminf(fmaxf(floorf(fn), -16777216.0f), 16777216.0f);
                fn = fn - fl;
                int32_t jn = j[k] + (int32_t)fl;
                if (fn >= 1.0f) { fn = 0.0f; jn += 1; }
                cfl |= live && !(fabsf(msf * nvx) < 1.0f);
                const bool bk = live && (!isfinite(nvx) || !isfinite(nvy) || !isfinite(nvz));
                bad |= bk;
                if (bk) jn = j[k], fn = f[k];  // keep the slot well-formed; the run is flagged
                bool l = false, r = false;
                if (periodic) {
                    if (jn < 0) jn += nc;
                    else if (jn >= nc) jn -= nc;
                    if (jn < 0 || jn >= nc) {
                        jn %= nc;
                        if (jn < 0) jn += nc;
                    }
                } else if (jn < 0) {
                    l = live;
                } else if (jn >= nc) {
                    r = live;
                }
                n_left += l;
                n_right += r;
                j[k] = (!live || l || r) ? kDeadCell : jn;
                f[k] = fn;
                vx[k] = nvx;
                vy[k] = nvy;
                vz[k] = nvz;
                if (j[k] >= 0) {
                    key[k] = j[k];
                    w1[k] = (unsigned long long)rintf(fn * 4294967296.0f);
                    if (test) {
                        const uint4 u = draw(pid[k], step, 0, key0, key1);
                        cand[k] = (unsigned long long)u.x < T;
                    }
                }
            }
            // ---- stores (no reads after this point in the tile touch these arrays)
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                if (o < rem && lv[k]) {
                    stream_st(&Xt[o], f[k]);
                    stream_st(&CELLt[o], j[k]);
                    stream_st(&VXt[o], vx[k]);
                    stream_st(&VYt[o], vy[k]);
                    stream_st(&VZt[o], vz[k]);
                }
            }
            // ---- rare events: wall losses, flags
            left = n_left > 0;
            right = n_right > 0;
            if (ballot(left) | ballot(right) | ballot(cfl) | ballot(bad)) {
                SegDyn *sd = d.segd + seg;
                InstDyn *idn = d.instd + inst;
                const unsigned long long ml = ballot(left), mr = ballot(right);
                int sl = n_left, sr = n_right;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    sl += __shfl_xor(sl, o, 64);
                    sr += __shfl_xor(sr, o, 64);
                }
                if (lane == 0) {
                    if (ml) atomicAdd(&sd->absorbed_step[0], (uint32_t)sl);
                    if (mr) atomicAdd(&sd->absorbed_step[1], (uint32_t)sr);
                }
                wave_or(&idn->status, PIC_ST_CFL, cfl);
                wave_or(&idn->status, PIC_ST_NONFINITE, bad);
            }
            // ---- candidates and deposit through LDS
            if (MCC) {
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                    queue_candidate(d, cand[k], (uint32_t)(tb + o), seg, inst, vx[k], vy[k], vz[k], pid[k], wn);
                }
            }
            if (DEP) {
                deposit_accumulate<NP>(L.wdep[wave], S, key, w1, dlo, dspan);
                dS = S;
                if (!d.late_flush && dspan > 0) {  // uniform
                    deposit_flush(L.wdep[wave], S, dlo, dspan);
                    dspan = 0;
                }
            }
        }
        // the block's next tile, from wave 0
        if (w0) {
            const int64_t i = tile_next(Q);
            const int64_t n = i >= 0 ? live_tile<kSegLds>(L, d, (uint32_t)i, lhint) : -1;
            if (lane_id() == 0) s_next[par] = n;
        }
        __syncthreads();
        t = uniform_i64(s_next[par]);
        par ^= 1;
    } while (t >= 0);
    else if (w0) (void)tile_next(Q);  // (no tile for this block: its counter still counts it done)
    if (DEP && dspan > 0) deposit_flush(L.wdep[wave], dS, dlo, dspan);
    if (MCC) flush_candidates(d, wn);
    if constexpr (MCC && COLL) collide_own_region(L, d, wn);
}

// ---------------------------------------------------------------------------
// FP64 form: double x in cells, double v; the same arithmetic as the FP64
// reference, operation by operation (no contraction, explicit fma in the gather)
// ---------------------------------------------------------------------------
// (held to 128 VGPRs, four waves per SIMD, with a 1024-block grid: the
// compiler spills one to three 4-byte values to scratch; at its free choice
// of 146 VGPRs the mover ran three waves per SIMD and the step 1.7% slower)
template <bool DEP, bool MCC, int NP, bool COLL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void push_f64_kernel(Dev d)
{
    __shared__ PushLds L;
    push_lds_init(L, d, true);
    const int cur = d.glob->cur_set;
    double *__restrict__ X = (double *)d.x[cur];
    double *__restrict__ VX = (double *)d.vx[cur];
    double *__restrict__ VY = (double *)d.vy[cur];
    double *__restrict__ VZ = (double *)d.vz[cur];
    const uint32_t *__restrict__ IDL = d.id_lo[cur];
    const uint32_t *__restrict__ IDH = d.id_hi[cur];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    uint32_t wn = 0;  // this wave's candidates so far (uniform)

    int hint = 0;  // segment of the previous tile
    // the constants of the segment of the previous tile, kept across tiles
    int cseg = -1;
    const double *__restrict__ acc = nullptr;
    unsigned long long *__restrict__ S = nullptr;
    double L_ = 0.0;
    bool periodic = false;
    double tx = 0.0, ty = 0.0, sx = 0.0, sy = 0.0, ms = 0.0, hk = 0.0;
    uint32_t key0 = 0, key1 = 0;
    unsigned long long T = 0;
    int inst = 0;
    long long step = 0;
    const uint32_t n_live = d.n_seg <= kSegLds ? live_tiles_init<kSegLds>(L, d) : (uint32_t)d.n_tiles;
    TileQueue Q;
    tile_queue_init(Q, d, n_live);
    int lhint = 0;  // segment of the previous live tile
    __shared__ int64_t s_next[2];  // the block's next tile, by parity of its tiles
    int par = 0;
    const int q = wave;  // the wave's part of each tile
    const bool w0 = __builtin_amdgcn_readfirstlane(wave) == 0;
    int64_t t = blockIdx.x < n_live ? live_tile<kSegLds>(L, d, blockIdx.x, lhint) : -1;
    if (t >= 0) do {
        int64_t tile0, base, count;
        uint32_t flg;
        const int seg = tile_seg(L, d, t, tile0, base, count, flg, hint);
        const int64_t t0 = (t - tile0) * (int64_t)kTile;
        // a subcycled species between its pushes keeps its positions (their
        // deposit is a launch of its own, deposit_kernel<true>)
        const bool work = t0 < count && !(d.n_seg > kSegLds && still(d, seg));
        // the tile in kPer / NP passes of NP chunks per wave (NP = kPer: one pass)
#pragma unroll 1
        for (int r0 = 0; work && r0 < kPer; r0 += NP) {
            const bool test = MCC && (flg & kFlgTest);
            const bool force = (flg & kFlgForce) != 0;

            double x[NP], vx[NP], vy[NP], vz[NP];
            unsigned long long pid[NP];
            const int64_t tb = base + t0;
            const uint32_t rem = (uint32_t)min(count - t0, (int64_t)kTile);
            double *__restrict__ Xt = X + tb;
            double *__restrict__ VXt = VX + tb;
            double *__restrict__ VYt = VY + tb;
            double *__restrict__ VZt = VZ + tb;
            const uint32_t *__restrict__ IDLt = IDL + tb;
            const uint32_t *__restrict__ IDHt = IDH + tb;
            if (rem == (uint32_t)kTile) {
                // a full tile: every load unconditional (see the FP32 form)
                if (test && !(flg & kFlgWide)) {
                    // every id below 2^32: the low words are the ids
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                        x[k] = stream_ld(&Xt[o]);
                        vx[k] = stream_ld(&VXt[o]);
                        vy[k] = stream_ld(&VYt[o]);
                        vz[k] = stream_ld(&VZt[o]);
                        pid[k] = stream_ld(&IDLt[o]);
                    }
                } else if (test) {
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                        x[k] = stream_ld(&Xt[o]);
                        vx[k] = stream_ld(&VXt[o]);
                        vy[k] = stream_ld(&VYt[o]);
                        vz[k] = stream_ld(&VZt[o]);
                        pid[k] = (unsigned long long)stream_ld(&IDLt[o]) |
                                 ((unsigned long long)stream_ld(&IDHt[o]) << 32);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                        x[k] = stream_ld(&Xt[o]);
                        vx[k] = stream_ld(&VXt[o]);
                        vy[k] = stream_ld(&VYt[o]);
                        vz[k] = stream_ld(&VZt[o]);
                        pid[k] = 0;
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                    x[k] = kDeadX;
                    vx[k] = vy[k] = vz[k] = 0.0;
                    pid[k] = 0;
                    if (o < rem) {
                        x[k] = stream_ld(&Xt[o]);
                        vx[k] = stream_ld(&VXt[o]);
                        vy[k] = stream_ld(&VYt[o]);
                        vz[k] = stream_ld(&VZt[o]);
                        if (test) {
                            pid[k] = stream_ld(&IDLt[o]);
                            if (flg & kFlgWide) pid[k] |= (unsigned long long)stream_ld(&IDHt[o]) << 32;
                        }
                    }
                }
            }
            if (w0 && r0 == 0) tile_grab(Q);  // the next tile, behind this one's loads
            // the segment's constants, read once the tile's loads are issued
            // (their scalar loads share a counter with the LDS reads that
            // address the tile: read first, the tile's loads would wait for them)
            if (r0 == 0 && seg != cseg) {
                const SegConst &sc = d.segc[seg];
                acc = d.acc64 + sc.sp * d.G + sc.gnode;
                S = d.S + sc.sp * d.G + sc.gnode;
                L_ = (double)sc.nc;
                periodic = (sc.bc == PIC_BC_PERIODIC);
                tx = sc.tx, ty = sc.ty, sx = sc.sx, sy = sc.sy;
                ms = sc.ms, hk = 0.5 * sc.ms;
                key0 = sc.key0, key1 = sc.key1;
                T = sc.T;
                inst = sc.inst;
                if (MCC) step = d.instd[inst].step;
                cseg = seg;
            }
            // the gather unpredicated (an empty slot reads node 0 and ignores it)
            double a0[NP], a1[NP], fr[NP];
            bool live[NP];
            int32_t jg[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                live[k] = x[k] >= 0.0;
                const double jd = floor(x[k]);
                jg[k] = live[k] ? (int32_t)jd : 0;
                fr[k] = live[k] ? x[k] - jd : 0.0;
            }
            if (force) {
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    a0[k] = acc[jg[k]];
                    a1[k] = acc[jg[k] + 1];
                }
            } else {
#pragma unroll
                for (int k = 0; k < NP; ++k) a0[k] = a1[k] = 0.0;
            }
            int key[NP];
            unsigned long long w1[NP];
            bool cand[NP];
            bool cfl = false, bad = false;
            int n_left = 0, n_right = 0;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                key[k] = -1;
                w1[k] = 0;
                cand[k] = false;
                // (dead lanes skip, unlike the FP32 form: with every lane running
                // the arithmetic the compiler spills two more values here, which
                // costs more than the waits before the stores that it saves)
                if (!live[k]) continue;
                const double a = fma(fr[k], a1[k] - a0[k], a0[k]);
                const double h = hk * a;
                const double mx = vx[k] + h, my = vy[k], mz = vz[k];
                const double px = mx - mz * ty;
                const double py = my + mz * tx;
                const double pz = mz + (mx * ty - my * tx);
                const double qx = mx - pz * sy;
                const double qy = my + pz * sx;
                const double qz = mz + (px * sy - py * sx);
                vx[k] = qx + h;
                vy[k] = qy;
                vz[k] = qz;
                double xn = x[k] + ms * vx[k];
                cfl |= !(fabs(ms * vx[k]) < 1.0);
                const bool bk = !isfinite(vx[k]) || !isfinite(vy[k]) || !isfinite(vz[k]);
                bad |= bk;
                if (bk) xn = x[k];
                bool l = false, r = false;
                if (periodic) {
                    if (xn < 0.0) xn += L_;
                    else if (xn >= L_) xn -= L_;
                    if (xn >= L_) xn -= L_;
                    if (!(xn >= 0.0 && xn < L_)) {  // displacement beyond one period (flagged)
                        xn = xn - L_ * floor(xn / L_);
                        if (!(xn >= 0.0 && xn < L_)) xn = 0.0;
                    }
                } else if (xn < 0.0) {
                    l = true;
                } else if (xn >= L_) {
                    r = true;
                }
                n_left += l;
                n_right += r;
                x[k] = (l || r) ? kDeadX : xn;
                if (x[k] >= 0.0) {
                    const double jn = floor(x[k]);
                    key[k] = (int)jn;
                    w1[k] = (unsigned long long)rint(ldexp(x[k] - jn, PIC_FRAC_BITS));
                    if (test) {
                        const uint4 u = draw(pid[k], step, 0, key0, key1);
                        cand[k] = (unsigned long long)u.x < T;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                if (o < rem && live[k]) {
                    stream_st(&Xt[o], x[k]);
                    stream_st(&VXt[o], vx[k]);
                    stream_st(&VYt[o], vy[k]);
                    stream_st(&VZt[o], vz[k]);
                }
            }
            const bool left = n_left > 0, right = n_right > 0;
            if (ballot(left) | ballot(right) | ballot(cfl) | ballot(bad)) {
                SegDyn *sd = d.segd + seg;
                InstDyn *idn = d.instd + inst;
                const unsigned long long ml = ballot(left), mr = ballot(right);
                int sl = n_left, sr = n_right;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    sl += __shfl_xor(sl, o, 64);
                    sr += __shfl_xor(sr, o, 64);
                }
                if (lane == 0) {
                    if (ml) atomicAdd(&sd->absorbed_step[0], (uint32_t)sl);
                    if (mr) atomicAdd(&sd->absorbed_step[1], (uint32_t)sr);
                }
                wave_or(&idn->status, PIC_ST_CFL, cfl);
                wave_or(&idn->status, PIC_ST_NONFINITE, bad);
            }
            if (MCC) {
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const uint32_t o = (uint32_t)((q * kPer + r0 + k) * 64 + lane);
                    queue_candidate(d, cand[k], (uint32_t)(tb + o), seg, inst, vx[k], vy[k], vz[k], pid[k], wn);
                }
            }
            if (DEP) deposit_tile<NP>(L, S, key, w1);
        }
        // the block's next tile, from wave 0
        if (w0) {
            const int64_t i = tile_next(Q);
            const int64_t n = i >= 0 ? live_tile<kSegLds>(L, d, (uint32_t)i, lhint) : -1;
            if (lane_id() == 0) s_next[par] = n;
        }
        __syncthreads();
        t = uniform_i64(s_next[par]);
        par ^= 1;
    } while (t >= 0);
    else if (w0) (void)tile_next(Q);  // (no tile for this block: its counter still counts it done)
    if (MCC) flush_candidates(d, wn);
    if constexpr (MCC && COLL) collide_own_region(L, d, wn);
}

// ---------------------------------------------------------------------------
// standalone deposit of the current positions (both forms)
// ---------------------------------------------------------------------------
// ONLY_STILL: just the tiles of subcycled species between their pushes
template <bool ONLY_STILL>
__global__ __launch_bounds__(kBlock) void deposit_kernel(Dev d)
{
    __shared__ PushLds L;
    push_lds_init(L, d);
    const int cur = d.glob->cur_set;
    int hint = 0;  // segment of the previous tile
    for (int64_t t = blockIdx.x; t < d.n_tiles; t += gridDim.x) {
        int64_t tile0, base, count;
        uint32_t flg;
        const int seg = tile_seg(L, d, t, tile0, base, count, flg, hint);
        const int64_t t0 = (t - tile0) * (int64_t)kTile;
        if (t0 >= count) continue;
        if (ONLY_STILL && !still(d, seg)) continue;
        deposit_positions(L, d, cur, d.segc[seg], base + t0, (uint32_t)min(count - t0, (int64_t)kTile));
    }
}

int push_grid(const Dev &d)
{
    // persistent-style grid, never more blocks than tiles: one block per
    // candidate region in use (the default the layout planned, or the grid
    // pic_set_mover chose, at most the layout's regions)
    return d.n_push_blocks;
}

template <bool DEP, bool MCC, int NP, bool COLL>
void launch_push_np(const Dev &d, hipStream_t st, dim3 grid)
{
    if (d.precision == PIC_FP64)
        hipLaunchKernelGGL((push_f64_kernel<DEP, MCC, NP, COLL>), grid, dim3(kBlock), 0, st, d);
    else
        hipLaunchKernelGGL((push_f32_kernel<DEP, MCC, NP, COLL>), grid, dim3(kBlock), 0, st, d);
}

template <bool DEP, bool MCC, bool COLL>
void launch_push_t(const Dev &d, hipStream_t st, dim3 grid, int chunks)
{
    if (chunks == kPer / 2) launch_push_np<DEP, MCC, kPer / 2, COLL>(d, st, grid);
    else launch_push_np<DEP, MCC, kPer, COLL>(d, st, grid);
}

hipError_t launch_push(const Dev &d, hipStream_t st, bool dep, bool mcc, bool subcycled, int chunks,
                       bool collide)
{
    const dim3 grid(push_grid(d));
    if (dep && mcc && collide) launch_push_t<true, true, true>(d, st, grid, chunks);
    else if (dep && mcc) launch_push_t<true, true, false>(d, st, grid, chunks);
    else if (dep) launch_push_t<true, false, false>(d, st, grid, chunks);
    else if (mcc && collide) launch_push_t<false, true, true>(d, st, grid, chunks);
    else if (mcc) launch_push_t<false, true, false>(d, st, grid, chunks);
    else launch_push_t<false, false, false>(d, st, grid, chunks);
    if (dep && subcycled) hipLaunchKernelGGL(deposit_kernel<true>, grid, dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_deposit(const Dev &d, hipStream_t st)
{
    hipLaunchKernelGGL(deposit_kernel<false>, dim3(push_grid(d)), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

}  // namespace picx
