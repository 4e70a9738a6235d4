/*
 * pic_layout.h -- C ABI of libpic_layout, the particle-layout study of the
 * mover: libpic's FP32 mover pass over one species (linear gather of the grid
 * acceleration, magnetised Boris push, advance, periodic re-entry, F = 32
 * fixed-point deposit, null-collision candidate test) with the particles
 * stored in one of four layouts.  Williams et al., arXiv 2404.10270, propose
 * vector-of-structs and array-of-structs movers as future work (Sec. 6) and
 * describe BIT1's "natural sorting", particles kept grouped by cell (Sec. 2);
 * this library measures those choices on one GPU.
 *
 *   PLS_SOA      structure of arrays (libpic's layout): cell i32, f f32,
 *                vx, vy, vz f32, id u64 -- 48 B moved per particle
 *   PLS_AOS      array of 32-byte structs {cell, f, vx, vy, vz, pad, id}
 *   PLS_AOSOA    blocks of 64 particles, structure of arrays inside a block
 *   PLS_CELLPAD  natural sorting: each cell owns `slack` slots (a multiple of
 *                64) and a count; the cell is the slot's, not stored.  A pass
 *                reads one buffer and writes every particle into its new
 *                cell's slots of the other (a regrouping by cell every step)
 *
 * Every layout computes the same particle results bit for bit (the order
 * of particles within a cell may differ for PLS_CELLPAD).  The deposit S
 * is the same u64 fixed-point sum in every layout.
 *
 * Ownership.  All buffers are device memory owned by the caller; `work`
 * holds the layout's particle storage (size from pls_work_bytes, 256-byte
 * aligned) and is not used by any other call.  Calls enqueue on `stream`
 * (a hipStream_t; NULL = the null stream) and do not synchronise.
 * Errors.  A negative return value before any work is enqueued: -1 bad
 * argument or layout, -3 a HIP call failed.  A PLS_CELLPAD cell whose slots
 * overflow drops the particle and flags the work buffer; pls_store then
 * returns -4.  Candidates are counted per block in the work buffer and
 * reported by pls_store.
 */
#ifndef PIC_LAYOUT_H
#define PIC_LAYOUT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { PLS_SOA = 0, PLS_AOS = 1, PLS_AOSOA = 2, PLS_CELLPAD = 3, PLS_N_LAYOUTS = 4 };

/* the particles of one species in libpic's FP32 form (device pointers) */
typedef struct {
    int32_t *cell;   /* cell index, 0 <= cell < nc */
    float *f;        /* in-cell offset in [0, 1) */
    float *vx, *vy, *vz;  /* cells per step */
    uint64_t *id;
} pls_soa;

typedef struct {
    int32_t nc;      /* cells (periodic) */
    int32_t slack;   /* PLS_CELLPAD: slots per cell, a multiple of 64 */
    float tx, ty, sx, sy;  /* Boris rotation: t = (q/m) B dt/2 (cos th, sin th), s = 2t/(1+|t|^2) */
    uint32_t key0, key1;   /* Philox key of the candidate test */
    uint64_t T;      /* candidate threshold floor(P 2^32) */
    const float *acc;      /* grid acceleration [nc+1], cells/step^2 */
    uint64_t *S;     /* deposit [nc+1], added to */
} pls_params;

/* bytes of the work buffer for n particles */
int pls_work_bytes(int layout, int64_t n, int32_t nc, int32_t slack, uint64_t *bytes);

/* copy n particles (PLS_CELLPAD: any order) from `in` into the layout */
int pls_load(int layout, const pls_soa *in, int64_t n, int32_t nc, int32_t slack, void *work,
             void *stream);

/* one mover pass at step `step` (keys the candidate draws); PLS_CELLPAD
 * alternates its two buffers: pass k reads buffer k mod 2 */
int pls_step(int layout, const pls_params *p, int64_t n, int64_t pass, int64_t step, void *work,
             void *stream);

/* copy the particles out (PLS_CELLPAD: after `passes` passes, grouped by
 * cell); *n_out receives the count copied and *n_cand the candidates of all
 * passes.  Synchronises the stream. */
int pls_store(int layout, void *work, int64_t n, int32_t nc, int32_t slack, int64_t passes,
              pls_soa *out, int64_t *n_out, uint64_t *n_cand, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PIC_LAYOUT_H */
