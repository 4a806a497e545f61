// launch.hpp -- host-side launch wrappers of the GRNND kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grnnd.h"

namespace grnnd {

// One collection of a batched build: its vertices are [base, base + n) of
// the concatenated points, its ids inside the batch are base + local id, and
// its random draws use its own seed on local ids, so that every collection's
// result equals its build alone. out_adj / out_keys: its output rows.
struct SegInfo {
  int64_t base;
  int64_t n;
  uint64_t seed;
  int32_t* out_adj;
  float* out_keys;
  int64_t pad;
};
static_assert(sizeof(SegInfo) == 48, "segment record layout");

// Segment of every vertex of a batched build; vseg == nullptr for a single
// collection (base 0, the launch's n and seed).
struct SegMap {
  const uint16_t* vseg;
  const SegInfo* segs;
};

struct VSeg {
  uint64_t seed;
  int64_t base, n;
};

__device__ __forceinline__ VSeg vseg_of(const SegMap& M, int64_t v, uint64_t seed, int64_t n) {
  if (!M.vseg) return VSeg{seed, 0, n};
  const SegInfo& s = M.segs[M.vseg[v]];
  return VSeg{s.seed, s.base, s.n};
}

// Where a round or reverse pass puts the items it emits (see RoundArgs).
struct ItemSink {
  uint2* own;        // n x R: (cand, key bits) kept by each vertex
  int32_t* nown;     // n
  uint2* bkt;        // n x bcap: items from other vertices
  int32_t bcap;
  uint32_t* cnt;     // n: items sent to each vertex so far
  uint4* ovf;        // overflow list: (dest, slot - bcap, cand, key bits)
  uint32_t* ovf_n;   // its length
};

// Arguments of the candidate round (update round or output pass).
struct RoundArgs {
  const float* X;  // points, row stride ld floats, 16-byte aligned rows
  int64_t n;
  int32_t d, d4, ld;
  int32_t R;
  const int32_t* in_ids;
  const float* in_keys;
  // update round: one item per candidate. The items v keeps (survivors) go
  // to the head of v's own row own[v * R ...], their number to nown[v]; an
  // item for another vertex x takes slot s = cnt[x]++ and goes to x's bucket
  // bkt[x * bcap + s] when s < bcap, else to the overflow list
  // ovf[(*ovf_n)++] = (x, s - bcap, cand, key bits)
  ItemSink items;
  // output pass
  int32_t* out_adj;
  float* out_keys;
  uint64_t seed;
  uint32_t round;
  int32_t order;
  int32_t x3;       // FP32 tiles of the grouped kernels in the three-product BF16 form
  int32_t defer;    // redirect keys that the tile does not give exactly are left to
                    // the merge (sent as kDeferredKey) instead of computed here
  float mcoef;      // tile error margin per unit of squared norm (grouped kernels)
  float mcoef_f32;  // the same for the FP32 matrix-core tile of the one-pool kernel
  const float* zero16;  // 16 zero bytes (fills the padding of LDS rows)
  unsigned long long* statp;
  // vertex lists from the classification pass: compact pools (valid entries
  // first) of at most 16, at most 32 and at most 64 entries, and any other
  // pool, with lengths vcount[0..3]
  const int32_t* vlist_s;
  const int32_t* vlist_m;
  const int32_t* vlist_l;
  const int32_t* vlist_b;
  const uint32_t* vcount;
  // narrow distance tile (prec != GRNND_PREC_FP32): the narrow copy of
  // x - c (ldr elements per row), FP8 row scales, per-row rounding error and
  // norm of x - c
  int32_t prec;
  const void* Xr;
  int64_t ldr;
  const float* rscale;
  const float2* rinfo;
  // per row flags (nullable; set for FP32, BF16 and FP16 tiles): bit 0 when
  // every element is an integer, bit 1 when every element is a BF16 value.
  // Two integer rows held exactly by the tile's copy (always for FP32;
  // rounding error 0 for a narrow copy) and with squared norms below 2^22
  // have an exact tile entry, equal to their canonical distance. An FP32
  // tile over rows that are all BF16 values needs no low-part products.
  const uint8_t* rexact;
  // the AND and the OR of every row's flags (set with rexact): when they are
  // equal every row has the same flags, and a wave reads them here instead
  // of one random byte per candidate
  const uint32_t* rsum;
  SegMap seg;  // collections of a batched build (arrival-order hashes)
};

struct InitArgs {
  const float* X;
  int64_t n;
  int32_t d, d4, ld;
  int32_t R, S;
  uint64_t seed;
  int32_t* out_ids;
  float* out_keys;
  uint32_t* cnt;  // nullable: zeroed for the first round
  const float* zero16;
  unsigned long long* statp;
  SegMap seg;  // draws stay inside each collection of a batched build
};

struct ReverseArgs {
  int64_t n;
  int32_t R;
  const int32_t* in_ids;
  const float* in_keys;
  uint64_t seed;
  uint32_t t1;
  int32_t mtab[65];  // floor(rho * k) for k = 0..64
  int32_t nearest;   // sample the nearest entries instead of the hash-first
  ItemSink items;
  unsigned long long* statp;
  SegMap seg;
};

// Merge of every vertex's items into its new pool.
struct MergeArgs {
  int64_t n;
  int32_t R;
  // the points (rows of ld floats, d4 float4 groups) and metric, for the
  // keys of deferred items (kDeferredKey)
  const float* X;
  int64_t ld;
  int32_t d4;
  int32_t metric;
  int32_t deferred;  // nonzero when the round may have left keys to the merge
  ItemSink items;
  uint32_t* off;     // n: start of each vertex's overflow items in seg (set where it has any)
  uint2* seg;        // overflow items grouped by destination
  uint32_t* cursor;  // [0] seg cursor, [5..8] merge list lengths
  uint4* mlist;      // 4 x n: (destination, kept, received, overflow start) by
                     // merge width (16, 32, 64, more)
  int32_t* out_ids;
  float* out_keys;
  unsigned long long* statp;
  // per destination: class of its new pool (0: at most 16 entries, 1: at
  // most 32, 2: more); the next round's classification reads it instead of
  // the pool rows
  uint8_t* pool_cls;
  // nonzero when every item sent to a vertex x with candidate c carries the
  // canonical distance d(x, c) bit for bit (the pool the round read was
  // written by this library in the same call): equal candidates then carry
  // equal keys
  int32_t canon;
};

struct SearchArgs {
  const float* X;
  int64_t n;
  int32_t d, d4, ld;
  int32_t metric;
  const int32_t* adj;
  int32_t R;
  int64_t entry;
  const float* Q;
  int32_t ldq;
  int64_t nq;
  int32_t k, L;
  int32_t* out_ids;
  float* out_keys;
  const float* zero16;
  const int64_t* entry_dev;  // non-null: the entry is read from here on the device
};

// Scratch of the medoid (byte offsets inside the region launch_medoid gets).
struct MedoidLayout {
  int nb;         // row blocks of the column sums
  int64_t chunk;  // rows per block
  size_t part_off, mean_off, dist_off, best_off, total;
};
MedoidLayout medoid_layout(int64_t n, int32_t d);
// *out (device int64) = the approximate medoid of X (n x d, row stride d).
hipError_t launch_medoid(const float* X, int64_t n, int32_t d, void* scratch, int64_t* out,
                         hipStream_t s);

// Dynamic LDS bytes of the round / init kernels for pool capacity R.
size_t round_lds_bytes(int R, int d);
size_t search_lds_bytes(int R, int d);

// Tile probe over nv candidate sets (see grnnd_tile_probe); uses X, n, d,
// d4, ld, R, mcoef and the narrow-tile fields of a.
hipError_t launch_tile_probe(const RoundArgs& a, int metric, const int32_t* ids, int64_t nv,
                             float* out_tile, float* out_band, float* out_canon, hipStream_t s);

// rexact[v]: bit 0 when row v of X (n x d, stride ld) holds only integers,
// bit 1 when it holds only BF16 values; rsum[0] and rsum[1]: the AND and the
// OR of all rows' flags.
hipError_t launch_rowflags(const float* X, int64_t n, int32_t d, int32_t ld, uint8_t* rexact,
                           uint32_t* rsum, hipStream_t s);

hipError_t launch_clear(uint32_t* cnt, int64_t n, uint32_t* cursor,
                        unsigned long long* statp, float* zero16, hipStream_t s);
hipError_t launch_pad_copy(const float* X, int64_t n, int32_t d, float* Xp, int32_t ldp,
                           hipStream_t s);
hipError_t launch_init(const InitArgs& a, int metric, hipStream_t s);
hipError_t launch_classify(const int32_t* ids, const uint8_t* pool_cls, const int32_t* order,
                           int64_t n, int32_t R, int32_t* const (&lists)[4], uint32_t* counts,
                           hipStream_t s);
// Narrow copy of the points for a BF16 / FP16 / FP8 tile (see quant.hip):
// part (256 x d floats) and center (d floats) are scratch for L2.
hipError_t launch_quantize(const float* X, int64_t n, int32_t d, int32_t ld, int metric, int prec,
                           float* part, float* center, void* Xr, int32_t ldr, float* rscale,
                           float2* rinfo, hipStream_t s);
// Locality order of the vertices (order[0..n)), from Voronoi cells of
// sampled pivots; cell (n bytes) and hist (kOrderPivots words) are scratch.
hipError_t launch_locality_order(const float* X, int64_t n, int32_t ld, uint64_t seed,
                                 uint8_t* cell, uint32_t* hist, int32_t* order, hipStream_t s);
hipError_t launch_round(const RoundArgs& a, int metric, bool final_pass, bool compact_pools,
                        hipStream_t s);
hipError_t launch_reverse(const ReverseArgs& a, hipStream_t s);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s);
hipError_t launch_stats_reduce(const unsigned long long* statp, uint64_t* dev_stats,
                               hipStream_t s);

// Segment table of a batched build, passed by value (at most kMaxSegs).
constexpr int kMaxSegs = 64;
struct SegTable {
  int32_t count;
  SegInfo seg[kMaxSegs];
};
// Writes the table to segs and every vertex's segment to vseg.
hipError_t launch_seg_fill(const SegTable& t, int64_t n, SegInfo* segs, uint16_t* vseg,
                           hipStream_t s);
// Output rows of every collection from the batch's rows (ids made local).
hipError_t launch_seg_split(const int32_t* adj, const float* keys, int64_t n, int32_t R,
                            const SegMap& m, hipStream_t s);
hipError_t launch_search(const SearchArgs& a, hipStream_t s);
// Verifies that a pool is canonical; *first_bad receives the smallest
// (row << 3 | code) of a violation, ~0 if there is none.
hipError_t launch_check_pool(const float* X, int64_t ld, int d4, int64_t n, int32_t R,
                             int32_t metric, const int32_t* ids, const float* keys,
                             unsigned long long* first_bad, hipStream_t s);

}  // namespace grnnd
