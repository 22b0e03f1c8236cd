// Device-side pieces of the bucketed path shared by its kernels
// (bucket_path.hip) and by the resident-simulation kernels (resident.hip):
// the bucket map, the boxes, the other-axis quantisation and the offsets
// through which the sweep finds each bucket's records.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace ddm {

// Buckets are the cells of a grid: nx columns by the swept axis' lower
// coordinate, each cut into ny rows by axis 1's lower coordinate (ny = 1:
// plain slabs of the swept axis).  Cell (column a, row c) is bucket
// a * ny + c, so a column's cells are consecutive; buckets from nx * ny to
// nb - 1 stay empty.
struct BucketParams {
  float vmin;        // column map of the swept axis' lower coordinate
  float scale;
  uint32_t nb;
  uint32_t valid;
  float qmin[2];     // 16-bit quantisation of the other axes (pre-filter);
  float qscale[2];   // see quant_t for the two forms of the map
  uint32_t nx, ny;   // columns, rows per column
  float vmin1;       // row map of axis 1's lower coordinate (ny > 1)
  float scale1;
  // the input axis swept (axis 0 of the boxes as the kernels see them; the
  // others follow in input order); kept in the first 64 bytes with the
  // fields every sweep workgroup reads first
  uint32_t axis;
  // bit k set: axis k + 1 is quantised on its encoded coordinate
  uint32_t qenc;
  // d >= 3: the axis (1 or 2) whose quantised bounds form the pre-filter word
  uint32_t qaxis;
  // split buckets (slabs only): if not null, column a of the map above became
  // the buckets split[a].x .. split[a].x + split[a].y - 1, by a map linear in
  // the encoded coordinate from split[a].z with scale __uint_as_float(split[a].w)
  const uint4 *split;
};

// bucket(x) = clamp(floor((x - vmin) * scale), 0, nb - 1): monotone
// non-decreasing in x, so a region whose lower coordinate falls in a later
// bucket starts strictly after every region of an earlier one.
__device__ __forceinline__ uint32_t bucket_of(float x, float vmin, float scale, uint32_t nb) {
  float t = (x - vmin) * scale;
  t = fminf(fmaxf(t, 0.0f), (float)(nb - 1));
  return (uint32_t)t;
}

// A device pointer as a pointer into the global address space.  Row
// pointers reach the kernels inside structures, where the compiler cannot
// tell their address space and reads them with generic (flat) loads, which
// also count against the LDS counter: every wait for an LDS result (the
// cursor atomics of the scatter, say) would then wait for the rows in flight.
template <typename T>
__device__ __forceinline__ const T __attribute__((address_space(1))) *global_ptr(const T *p) {
  return (const T __attribute__((address_space(1))) *)p;
}

// The bucket of swept-axis coordinate x in column a of a split map: the
// column's first bucket plus floor((enc(x) - z) * scale), clamped to the
// column's buckets.  Encoding, subtraction (clamped at 0), conversion to
// float and scaling are all non-decreasing, so the map stays monotone and
// the columns stay consecutive segments.
__device__ __forceinline__ uint32_t split_of(float x, uint32_t a, const uint4 *__restrict__ split) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const v4u r = global_ptr(reinterpret_cast<const v4u *>(split))[a];
  if (r.y <= 1u) return r.x;
  const long long off = (long long)encode_coord(x) - (long long)r.z;
  float t = (float)(off > 0 ? off : 0ll) * __uint_as_float(r.w);
  t = fminf(t, (float)(r.y - 1u));
  return r.x + (uint32_t)t;
}

template <int D>
struct Box {
  float lo[D];
  float hi[D];
};

// The grid cells a box overlaps: columns [a0, a1] (of its swept-axis
// bounds) by rows [c0, c1] (of its axis-1 bounds).  Its record goes to cell
// (a0, c0); the cells (a0, c) for c > c0 get copies as ordinary records
// (within the column the box keeps its own swept-axis position); cells of
// later columns get boundary-state copies.  A pair is found in the column
// of its later swept-axis lower bound (as with slabs) and counted in the
// row that holds the larger of its two axis-1 lower bounds; both boxes are
// present in that cell, since the maps are monotone.
template <int D>
struct Cells {
  uint32_t a0, a1, c0, c1;
};

// Kernels take the per-box work in two forms, chosen once per workgroup:
// GRID = false for slabs (ny = 1, rows known to be 0 at compile time) and
// GRID = true for a grid.
template <bool GRID>
struct GridTag {
  static constexpr bool value = GRID;
};

template <bool GRID>
__device__ __forceinline__ uint32_t cell_index(uint32_t a, uint32_t c, const BucketParams &p) {
  return GRID ? a * p.ny + c : a;
}

// The cell of a box's record and its row: (a0 * ny + c0, c0).
template <int D, bool GRID>
__device__ __forceinline__ uint2 home_of(const Box<D> &b, const BucketParams &p) {
  uint32_t a = bucket_of(b.lo[0], p.vmin, p.scale, p.nx);
  if (p.split) a = split_of(b.lo[0], a, p.split);  // slabs only (ny = 1)
  uint32_t c = 0u;
  if (GRID && D >= 2) c = bucket_of(b.lo[1 % D], p.vmin1, p.scale1, p.ny);
  return make_uint2(cell_index<GRID>(a, c, p), c);
}

template <int D, bool GRID>
__device__ __forceinline__ Cells<D> cells_of(const Box<D> &b, const BucketParams &p) {
  Cells<D> c;
  c.a0 = bucket_of(b.lo[0], p.vmin, p.scale, p.nx);
  c.a1 = bucket_of(b.hi[0], p.vmin, p.scale, p.nx);
  if (p.split) {  // slabs only (ny = 1)
    c.a0 = split_of(b.lo[0], c.a0, p.split);
    c.a1 = split_of(b.hi[0], c.a1, p.split);
  }
  c.c0 = c.c1 = 0u;
  if (GRID && D >= 2) {
    c.c0 = bucket_of(b.lo[1 % D], p.vmin1, p.scale1, p.ny);
    c.c1 = bucket_of(b.hi[1 % D], p.vmin1, p.scale1, p.ny);
  }
  return c;
}

// Error bits and emptiness of one box.  A half-open box with lo == hi on
// some axis is empty; a closed one never is (lo == hi is a point).
template <int D>
__device__ __forceinline__ uint32_t box_errors(const Box<D> &b, bool &empty, uint32_t closed) {
  uint32_t err = 0;
  empty = false;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float l = b.lo[k], h = b.hi[k];
    if (l != l || h != h) err |= kErrNaN;
    if (l > h) err |= kErrOrder;
    if (l == h && !closed) empty = true;
  }
  return err;
}

// Conservative quantisation of a coordinate of another axis onto 16 bits by
// a monotone map t = clamp(quant_t(x), 0, 65535): lower bounds round down,
// upper bounds round up, so two boxes that overlap on that axis also overlap
// after quantisation.  Quantised bounds only serve the sweep's pre-filter;
// survivors are tested on the exact coordinates.  The map is linear in the
// coordinate, (x - qmin) * qscale, or, for an axis whose boxes spread over
// many orders of magnitude, linear in its encoded coordinate (about
// logarithmic in |x|): (enc(x) - e0) * qscale, e0 the bits held in qmin and
// differences below 0 taken as 0.  Encoding, subtraction, conversion to
// float and scaling are all non-decreasing, so either form is monotone.
__device__ __forceinline__ float quant_t(float x, float qmin, float qs, bool enc) {
  if (enc) {
    const uint32_t e = encode_coord(x), e0 = __float_as_uint(qmin);
    return (float)(e > e0 ? e - e0 : 0u) * qs;
  }
  return (x - qmin) * qs;
}

__device__ __forceinline__ uint32_t quant_lo(float x, float qmin, float qs, bool enc) {
  float t = quant_t(x, qmin, qs, enc);
  t = fminf(fmaxf(t, 0.0f), 65535.0f);
  return (uint32_t)t;
}

__device__ __forceinline__ uint32_t quant_hi(float x, float qmin, float qs, bool enc) {
  float t = quant_t(x, qmin, qs, enc);
  t = fminf(fmaxf(t, 0.0f), 65535.0f);
  return (uint32_t)ceilf(t);
}

// Axis 1 on a grid (ny > 1) is quantised over the record's own row: every
// record of a cell, copies included, is written for that cell's row, and
// t = ((x - vmin1) * scale1 - row) * 65535 is as monotone as the map above,
// so the pre-filter stays conservative while keeping its resolution inside
// a row (bounds beyond the row clamp to its ends).
__device__ __forceinline__ uint32_t quant1_lo(float x, const BucketParams &p, uint32_t row) {
  if (p.ny <= 1) return quant_lo(x, p.qmin[0], p.qscale[0], p.qenc & 1u);
  float t = ((x - p.vmin1) * p.scale1 - (float)row) * 65535.0f;
  t = fminf(fmaxf(t, 0.0f), 65535.0f);
  return (uint32_t)t;
}

__device__ __forceinline__ uint32_t quant1_hi(float x, const BucketParams &p, uint32_t row) {
  if (p.ny <= 1) return quant_hi(x, p.qmin[0], p.qscale[0], p.qenc & 1u);
  float t = ((x - p.vmin1) * p.scale1 - (float)row) * 65535.0f;
  t = fminf(fmaxf(t, 0.0f), 65535.0f);
  return (uint32_t)ceilf(t);
}

// Word 3 of a region record in a cell of grid row ``row``: the 16-bit
// lower | upper << 16 bounds of one other axis, axis 1 for d = 2 and axis
// p.qaxis (1 or 2) for d >= 3; 0 for d = 1.  Sixteen bits of one axis filter
// far better than seven of two: at the workloads' sizes a box's side is a
// few 65536ths of an axis, while a 128th holds hundreds of boxes, so one
// sharp axis rejects about ten times more candidates (seventy times more on
// clustered inputs, where axes 1 and 2 follow axis 0 within a cluster).  On
// a grid, whose rows already bound axis 1, the plan filters on axis 2.
template <int D>
__device__ __forceinline__ uint32_t qword_of(const Box<D> &b, const BucketParams &p,
                                             uint32_t row) {
  if (D == 2 || (D >= 3 && p.qaxis != 2u))
    return quant1_lo(b.lo[1 % D], p, row) | (quant1_hi(b.hi[1 % D], p, row) << 16);
  if (D >= 3)
    return quant_lo(b.lo[2 % D], p.qmin[1], p.qscale[1], p.qenc & 2u) |
           (quant_hi(b.hi[2 % D], p.qmin[1], p.qscale[1], p.qenc & 2u) << 16);
  return 0u;
}

// Where the sweep finds bucket j's records and boundary-state entries.
//
// Packed layout (a matching call): the one prefix sum over [bucket sizes |
// boundary-state sizes | 0] (2 nb + 1 entries, buckets numbered over all
// instances) gives S[j], the first record slot of bucket j, S[nb], the
// number of records, and S[nb + j] - S[nb], the first boundary-state entry
// of bucket j (j <= nb).  Block k's first slot in bucket j is S[j] plus the
// block-major prefix written by bk_colscan_kernel.
//
// Slab layout (a resident simulation, cnt non-null): bucket j owns the
// fixed slots [j * cap, (j + 1) * cap) of which the first cnt[j] hold
// records, and [j * bs_slab, (j + 1) * bs_slab) of the boundary-state
// records, of which the first bs_cnt[j] are filled (a count above bs_slab
// means some did not fit).
struct Offsets {
  const uint32_t *S;
  uint32_t nb;  // buckets over all instances
  const uint32_t *cnt = nullptr, *bs_cnt = nullptr;
  uint32_t cap = 0, bs_slab = 0;
  // packed layout: every instance's grid, and the record buffer's capacity
  // (copies into later rows make the records more than the regions; slots
  // from rec_cap on are not written and the sweep sends the call back)
  const BucketParams *P = nullptr;
  uint32_t rec_cap = 0;
  __device__ uint32_t bs_begin(uint32_t j) const { return S[nb + j] - S[nb]; }
};

}  // namespace ddm
