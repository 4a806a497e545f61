// api.cpp -- C ABI of the GRNND library (see include/grnnd.h).
//
// Host orchestration only: argument checks, workspace carving, and the launch
// schedule of Alg. 3 (init; T1 x (T2 update rounds; reverse sampling unless
// last); output pass). Everything is enqueued on the caller's stream with no
// host synchronisation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "grnnd.h"
#include "launch.hpp"
#include "common.hpp"

using namespace grnnd;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

namespace grnnd {
// Sets the calling thread's last-error text (used by the build server).
int set_error(int code, const char* msg) {
  g_err = msg;
  return code;
}
}  // namespace grnnd

namespace {

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(GRNND_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

// ------------------------------------------------------------ kernel timing
struct ProfRec {
  int kind;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;

// Brackets one launch with events when timing is enabled.
struct ProfScope {
  ProfRec r{};
  bool on = false;
  hipStream_t s;
  ProfScope(int kind, hipStream_t st) : s(st) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    if (hipEventCreate(&r.a) != hipSuccess) return;
    if (hipEventCreate(&r.b) != hipSuccess) {
      (void)hipEventDestroy(r.a);
      return;
    }
    r.kind = kind;
    on = hipEventRecord(r.a, s) == hipSuccess;
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(r.b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back(r);
  }
};

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int mfloor(float rho, int k) { return (int)std::floor((double)rho * (double)k); }

struct Ws {
  int32_t* pa_ids;
  float* pa_keys;
  int32_t* pb_ids;
  float* pb_keys;
  uint2* own;       // n x R kept items
  int32_t* nown;
  uint2* bkt;       // n x R received items (bucket capacity R)
  uint4* ovf;       // overflow list, n x R entries at most
  uint4* mlist;     // 4 x n merge-list entries
  uint32_t* cnt;
  uint32_t* off;
  uint2* seg;
  uint32_t* cursor;  // [0] seg cursor, [1..4] vertex-list lengths, [5..8] merge-list
                     // lengths, [9] overflow count
  int32_t* vlist_s;
  int32_t* vlist_m;
  int32_t* vlist_l;
  int32_t* vlist_b;
  uint8_t* pool_cls;
  int32_t* order;  // locality order of the vertices (built once per build)
  void* xr;        // narrow copy of x - c (narrow tiles only)
  int32_t ldr;     // its row length in elements (d rounded up to 32)
  float* rscale;   // FP8 row scales
  float2* rinfo;   // per row: rounding error and norm of x - c
  uint8_t* rexact;  // per row: integer-valued
  float* qpart;    // column-sum partials (256 x d)
  float* qcenter;  // the centre c
  uint8_t* cell;
  uint32_t* chist;
  unsigned long long* statp;
  float* zero16;
  unsigned long long* check;  // result slot of the pool check
  uint32_t* rsum;             // AND and OR of the row flags
  float* xpad;
  // batched builds: the concatenated points (rows of round_up(d, 4) floats),
  // the segment table and every vertex's segment
  float* xcat;
  SegInfo* segs;
  uint16_t* vseg;
  int32_t cap;
  size_t total;
};

// Carves the workspace; with base == nullptr only computes sizes. nseg > 0
// adds the areas of a batched build of nseg collections (n points in all).
Ws ws_layout(void* base, int64_t n, int32_t d, int32_t R, const grnnd_params& p,
             int32_t nseg = 0) {
  Ws W{};
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* ptr = base ? static_cast<char*>(base) + off : nullptr;
    off = align_up(off + bytes);
    return ptr;
  };
  const int64_t nR = n * R;
  // items that overflow their destination's bucket in one pass: at most one
  // per candidate sent elsewhere, so at most n * R
  W.cap = R;
  const int64_t ni = n * (int64_t)W.cap;
  W.pa_ids = reinterpret_cast<int32_t*>(take(nR * 4));
  W.pa_keys = reinterpret_cast<float*>(take(nR * 4));
  W.pb_ids = reinterpret_cast<int32_t*>(take(nR * 4));
  W.pb_keys = reinterpret_cast<float*>(take(nR * 4));
  W.own = reinterpret_cast<uint2*>(take(nR * 8));
  W.nown = reinterpret_cast<int32_t*>(take(n * 4));
  W.bkt = reinterpret_cast<uint2*>(take(nR * 8));
  W.ovf = reinterpret_cast<uint4*>(take(ni * 16));
  W.mlist = reinterpret_cast<uint4*>(take(n * 64));
  W.cnt = reinterpret_cast<uint32_t*>(take(n * 4));
  W.off = reinterpret_cast<uint32_t*>(take(n * 4));
  W.seg = reinterpret_cast<uint2*>(take(ni * 8));
  W.cursor = reinterpret_cast<uint32_t*>(take(kCursorWords * 4));
  W.vlist_s = reinterpret_cast<int32_t*>(take(n * 4));
  W.vlist_m = reinterpret_cast<int32_t*>(take(n * 4));
  W.vlist_l = reinterpret_cast<int32_t*>(take(n * 4));
  W.vlist_b = reinterpret_cast<int32_t*>(take(n * 4));
  W.pool_cls = reinterpret_cast<uint8_t*>(take(n));
  W.rexact = reinterpret_cast<uint8_t*>(take(n));
  W.order = reinterpret_cast<int32_t*>(take(n * 4));
  W.cell = reinterpret_cast<uint8_t*>(take(n));
  W.chist = reinterpret_cast<uint32_t*>(take((size_t)kOrderPivots * 4));
  W.statp = reinterpret_cast<unsigned long long*>(take((size_t)kStatSlots * kStatStride * 8));
  W.zero16 = reinterpret_cast<float*>(take(256));
  W.check = reinterpret_cast<unsigned long long*>(take(8));
  W.rsum = reinterpret_cast<uint32_t*>(take(8));
  if (nseg > 0) {
    W.xcat = reinterpret_cast<float*>(take((size_t)n * round_up(d, 4) * 4));
    W.segs = reinterpret_cast<SegInfo*>(take((size_t)nseg * sizeof(SegInfo)));
    W.vseg = reinterpret_cast<uint16_t*>(take((size_t)n * 2));
  }
  W.xpad = (d % 4 && nseg == 0) ? reinterpret_cast<float*>(take((size_t)n * round_up(d, 4) * 4))
                                : nullptr;
  if (p.precision != GRNND_PREC_FP32) {
    const size_t esz = p.precision == GRNND_PREC_FP8_E4M3 ? 1 : 2;
    W.ldr = round_up(d, 32);
    W.xr = take((size_t)n * W.ldr * esz);
    W.rscale = reinterpret_cast<float*>(take((size_t)n * 4));
    W.rinfo = reinterpret_cast<float2*>(take((size_t)n * 8));
    W.qpart = reinterpret_cast<float*>(take((size_t)256 * d * 4));
    W.qcenter = reinterpret_cast<float*>(take((size_t)d * 4));
  }
  W.total = off;
  return W;
}

size_t max_lds_bytes() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 65536;
  return (size_t)v;
}

int check_params(const grnnd_params& p, int32_t R) {
  if (p.S < 1 || p.S > R) return fail(GRNND_EINVAL, "S=%d must be in [1, R=%d]", p.S, R);
  if (p.T1 < 1 || p.T2 < 1) return fail(GRNND_EINVAL, "T1=%d, T2=%d must be >= 1", p.T1, p.T2);
  if (!(p.rho > 0.0f && p.rho < 1.0f)) return fail(GRNND_EINVAL, "rho=%g must be in (0,1)", p.rho);
  if (p.order < 0 || p.order > 2) return fail(GRNND_EINVAL, "order=%d unknown", p.order);
  if (p.precision < GRNND_PREC_FP32 || p.precision > GRNND_PREC_FP8_E4M3)
    return fail(GRNND_EINVAL, "precision=%d unknown", p.precision);
  if (p.reverse != GRNND_REVERSE_HASH && p.reverse != GRNND_REVERSE_NEAREST)
    return fail(GRNND_EINVAL, "reverse=%d unknown", p.reverse);
  if (p.check != 0 && p.check != 1) return fail(GRNND_EINVAL, "check=%d must be 0 or 1", p.check);
  return GRNND_OK;
}

int check_sizes(const float* points, int64_t n, int32_t d, int32_t metric, int32_t R) {
  if (!points) return fail(GRNND_EINVAL, "points is null");
  if (n < 2 || n >= (int64_t)1 << 31) return fail(GRNND_EINVAL, "n=%lld out of range", (long long)n);
  if (d < 1 || d > 4096) return fail(GRNND_EINVAL, "d=%d out of range [1, 4096]", d);
  if (metric != GRNND_METRIC_L2 && metric != GRNND_METRIC_IP)
    return fail(GRNND_EINVAL, "metric=%d unknown", metric);
  if (R < 1 || R > GRNND_MAX_R) return fail(GRNND_EINVAL, "R=%d out of range [1, 64]", R);
  if (d % 4 == 0 && (reinterpret_cast<uintptr_t>(points) & 15))
    return fail(GRNND_EINVAL, "points must be 16-byte aligned");
  const size_t lds = round_lds_bytes(R, round_up(d, 4));
  if (lds > max_lds_bytes())
    return fail(GRNND_ENOTSUP, "R=%d, d=%d needs %zu B of LDS per wave (limit %zu)", R, d, lds,
                max_lds_bytes());
  return GRNND_OK;
}

grnnd_params defaults(int32_t R, int32_t iters) {
  grnnd_params p;
  p.S = R;
  p.T1 = iters;
  p.T2 = 4;
  p.rho = 0.6f;
  p.order = GRNND_ORDER_DISORDERED;
  p.precision = GRNND_PREC_FP32;
  p.reverse = GRNND_REVERSE_HASH;
  p.check = 0;
  return p;
}

struct Ctx {
  const float* X;
  int32_t ld, d4;
  int64_t n;
  int32_t d, metric, R;
  grnnd_params p;
  Ws W;
  hipStream_t s;
  // true once a merge of this call has recorded which of the pools it wrote
  // are small; until then the classification reads the pool rows
  mutable bool lists_ready = false;
  // true once every row of the pool the next round reads was written by this
  // call (init or a merge): such rows are compact, so pool classes wider than
  // R allows are empty
  mutable bool compact = false;
  // locality order the round kernels walk their vertex lists in (null: by id)
  const int32_t* order = nullptr;
  // the narrow copy of the points has been made in this call
  mutable bool narrow_ready = false;
  // the integer-row flags have been computed in this call
  mutable bool rexact_ready = false;
  // collections of a batched build (vseg null: one collection)
  SegMap seg{nullptr, nullptr};
};

int setup(Ctx& c, const float* points, int64_t n, int32_t d, int32_t metric, int32_t R,
          const grnnd_params* pp, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_sizes(points, n, d, metric, R);
  if (rc) return rc;
  c.p = pp ? *pp : defaults(R, 1);
  rc = check_params(c.p, R);
  if (rc) return rc;
  const Ws need = ws_layout(nullptr, n, d, R, c.p);
  if (!ws) return fail(GRNND_EINVAL, "workspace is null");
  if (ws_bytes < need.total)
    return fail(GRNND_ENOSPACE, "workspace has %zu B, needs %zu B", ws_bytes, need.total);
  if (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1))
    return fail(GRNND_EINVAL, "workspace must be 256-byte aligned");
  if ((uint64_t)n * (uint64_t)need.cap >= ((uint64_t)1 << 32))
    return fail(GRNND_ENOTSUP, "n * items per vertex exceeds 2^32");
  c.W = ws_layout(ws, n, d, R, c.p);
  c.n = n;
  c.d = d;
  c.metric = metric;
  c.R = R;
  c.s = static_cast<hipStream_t>(stream);
  c.d4 = (d + 3) / 4;
  if (d % 4) {
    c.ld = 4 * c.d4;
    HIP_OK(launch_pad_copy(points, n, d, c.W.xpad, c.ld, c.s));
    c.X = c.W.xpad;
  } else {
    c.ld = d;
    c.X = points;
  }
  return GRNND_OK;
}

// Tile error coefficient per unit of squared norm for the FP32 accumulation
// over the padded row length (16 floats per FP32 step, 32 elements per
// narrow step).
// Rows of at least this many elements get FP32 tiles in the three-product
// BF16 form in the grouped kernels (shorter rows: the FP32 matrix cores).
constexpr int kX3MinD = 512;

bool use_x3(const Ctx& c) { return c.p.precision == GRNND_PREC_FP32 && c.d >= kX3MinD; }

// Rows of at least this many elements leave the redirect keys that the tile
// does not give exactly to the merge: computed in the round, each would
// gather both rows of its pair a second time, after the pool's other rows
// have pushed them out of L2; the merge reads the destination's row once for
// all of its items and skips candidates the destination already holds.
// Below it the round's own gathers overlap those reads well enough that
// moving them to a kernel of their own does not pay.
constexpr int kDeferMinD = 512;

// Tile margin per unit of squared norm. FP32 tiles on the FP32 matrix cores
// and narrow tiles: (2 len + 4) u over the padded row length len. The
// three-product form splits each row as x = hi + lo + e (hi = bf16(x),
// lo = bf16(x - hi), |e| <= 2^-16 |x|) and sums the exact BF16 products
// hi hi' + hi lo' + lo hi' in one chain, 3 len terms: (3 len + 4) u, plus
// the dropped terms lo lo' and those of e, below 3.1 * 2^-16 |x||x'| per
// element, covered by 2^-14. (Tiles whose rows are all BF16 values sum len
// exact products, within either bound.)
float margin_coef(const Ctx& c) {
  const double u = std::ldexp(1.0, -24);
  const bool fp32 = c.p.precision == GRNND_PREC_FP32;
  const int len = fp32 ? round_up(4 * c.d4, 16) : round_up(c.d, 32);
  const bool x3 = use_x3(c);
  const int m = x3 ? 3 * len + 4 : 2 * len + 4;
  const double t = x3 ? std::ldexp(1.0, -14) : 0.0;
  return (float)((c.metric == GRNND_METRIC_L2 ? 4.0 : 1.0) * (m * u + t));
}

float margin_coef_f32(const Ctx& c) {
  const double u = std::ldexp(1.0, -24);
  const int m = 2 * round_up(4 * c.d4, 16) + 4;
  return (float)((c.metric == GRNND_METRIC_L2 ? 4.0 : 1.0) * m * u);
}

// Makes the narrow copy of the points once per call (narrow tiles only).
int ensure_narrow(const Ctx& c) {
  if (c.p.precision == GRNND_PREC_FP32 || c.narrow_ready) return GRNND_OK;
  ProfScope ps(GRNND_PROF_INIT, c.s);
  HIP_OK(launch_quantize(c.X, c.n, c.d, c.ld, c.metric, c.p.precision, c.W.qpart, c.W.qcenter,
                         c.W.xr, c.W.ldr, c.W.rscale, c.W.rinfo, c.s));
  c.narrow_ready = true;
  return GRNND_OK;
}

ItemSink sink(const Ctx& c) {
  ItemSink k{};
  k.own = c.W.own;
  k.nown = c.W.nown;
  k.bkt = c.W.bkt;
  k.bcap = c.R;
  k.cnt = c.W.cnt;
  k.ovf = c.W.ovf;
  k.ovf_n = c.W.cursor + 9;
  return k;
}

// Integer-row flags for the exact redirect keys of FP32, BF16 and FP16 L2
// tiles.
int ensure_rexact(const Ctx& c) {
  if (c.p.precision == GRNND_PREC_FP8_E4M3 || c.rexact_ready) return GRNND_OK;
  if (c.metric != GRNND_METRIC_L2 && c.p.precision != GRNND_PREC_FP32) return GRNND_OK;
  ProfScope ps(GRNND_PROF_INIT, c.s);
  HIP_OK(launch_rowflags(c.X, c.n, c.d, c.ld, c.W.rexact, c.W.rsum, c.s));
  c.rexact_ready = true;
  return GRNND_OK;
}

void set_narrow(const Ctx& c, RoundArgs& a) {
  a.prec = c.p.precision;
  a.Xr = c.W.xr;
  a.ldr = c.W.ldr;
  a.rscale = c.W.rscale;
  a.rinfo = c.W.rinfo;
  a.rexact = c.rexact_ready ? c.W.rexact : nullptr;
  a.rsum = c.rexact_ready ? c.W.rsum : nullptr;
}

int do_update(const Ctx& c, const int32_t* in_ids, const float* in_keys, int32_t* out_ids,
              float* out_keys, uint64_t seed, uint32_t round) {
  int rc = ensure_narrow(c);
  if (rc) return rc;
  if ((rc = ensure_rexact(c))) return rc;
  RoundArgs a{};
  set_narrow(c, a);
  a.X = c.X;
  a.n = c.n;
  a.d = c.d;
  a.d4 = c.d4;
  a.ld = c.ld;
  a.R = c.R;
  a.in_ids = in_ids;
  a.in_keys = in_keys;
  a.items = sink(c);
  a.seed = seed;
  a.round = round;
  a.order = c.p.order;
  a.seg = c.seg;
  a.mcoef = margin_coef(c);
  a.mcoef_f32 = margin_coef_f32(c);
  a.x3 = use_x3(c) ? 1 : 0;
  a.defer = c.d >= kDeferMinD ? 1 : 0;
  a.zero16 = c.W.zero16;
  a.statp = c.W.statp;
  a.vlist_s = c.W.vlist_s;
  a.vlist_m = c.W.vlist_m;
  a.vlist_l = c.W.vlist_l;
  a.vlist_b = c.W.vlist_b;
  a.vcount = c.W.cursor + 1;
  {
    ProfScope ps(GRNND_PROF_UPDATE, c.s);
    int32_t* const lists[4] = {c.W.vlist_s, c.W.vlist_m, c.W.vlist_l, c.W.vlist_b};
    HIP_OK(launch_classify(in_ids, c.lists_ready ? c.W.pool_cls : nullptr, c.order, c.n, c.R,
                           lists, c.W.cursor + 1, c.s));
    HIP_OK(launch_round(a, c.metric, false, c.compact, c.s));
  }
  MergeArgs m{};
  m.n = c.n;
  m.R = c.R;
  m.X = c.X;
  m.ld = c.ld;
  m.d4 = c.d4;
  m.metric = c.metric;
  m.deferred = a.defer;
  m.items = sink(c);
  m.off = c.W.off;
  m.cursor = c.W.cursor;
  m.seg = c.W.seg;
  m.mlist = c.W.mlist;
  m.out_ids = out_ids;
  m.out_keys = out_keys;
  m.statp = c.W.statp;
  m.pool_cls = c.W.pool_cls;
  m.canon = c.compact ? 1 : 0;  // the pool read was written by this call
  {
    ProfScope ps(GRNND_PROF_MERGE, c.s);
    HIP_OK(launch_merge(m, c.s));
    c.lists_ready = true;
    c.compact = true;
  }
  return GRNND_OK;
}

int do_reverse(const Ctx& c, const int32_t* in_ids, const float* in_keys, int32_t* out_ids,
               float* out_keys, uint64_t seed, uint32_t t1) {
  ReverseArgs a{};
  a.n = c.n;
  a.R = c.R;
  a.in_ids = in_ids;
  a.in_keys = in_keys;
  a.seed = seed;
  a.t1 = t1;
  for (int k = 0; k <= 64; ++k) a.mtab[k] = mfloor(c.p.rho, k);
  a.nearest = c.p.reverse == GRNND_REVERSE_NEAREST ? 1 : 0;
  a.seg = c.seg;
  a.items = sink(c);
  a.statp = c.W.statp;
  {
    ProfScope ps(GRNND_PROF_REVERSE, c.s);
    HIP_OK(launch_reverse(a, c.s));
  }
  MergeArgs m{};
  m.n = c.n;
  m.R = c.R;
  m.X = c.X;
  m.ld = c.ld;
  m.d4 = c.d4;
  m.metric = c.metric;
  m.items = sink(c);
  m.off = c.W.off;
  m.cursor = c.W.cursor;
  m.seg = c.W.seg;
  m.mlist = c.W.mlist;
  m.out_ids = out_ids;
  m.out_keys = out_keys;
  m.statp = c.W.statp;
  m.pool_cls = c.W.pool_cls;
  m.canon = c.compact ? 1 : 0;  // the pool read was written by this call
  {
    ProfScope ps(GRNND_PROF_MERGE, c.s);
    HIP_OK(launch_merge(m, c.s));
    c.lists_ready = true;
    c.compact = true;
  }
  return GRNND_OK;
}

int do_init(const Ctx& c, int32_t S, uint64_t seed, int32_t* out_ids, float* out_keys) {
  InitArgs a{};
  a.X = c.X;
  a.n = c.n;
  a.d = c.d;
  a.d4 = c.d4;
  a.ld = c.ld;
  a.R = c.R;
  a.S = S;
  a.seed = seed;
  a.out_ids = out_ids;
  a.out_keys = out_keys;
  a.seg = c.seg;
  a.cnt = c.W.cnt;
  a.zero16 = c.W.zero16;
  a.statp = c.W.statp;
  {
    ProfScope ps(GRNND_PROF_INIT, c.s);
    HIP_OK(launch_init(a, c.metric, c.s));
  }
  c.compact = true;  // each row: its ids in (key, id) order, then -1 padding
  return GRNND_OK;
}

int do_final(const Ctx& c, const int32_t* in_ids, const float* in_keys, int32_t* out_adj,
             float* out_keys) {
  int rc = ensure_narrow(c);
  if (rc) return rc;
  if ((rc = ensure_rexact(c))) return rc;
  RoundArgs a{};
  set_narrow(c, a);
  a.X = c.X;
  a.n = c.n;
  a.d = c.d;
  a.d4 = c.d4;
  a.ld = c.ld;
  a.R = c.R;
  a.in_ids = in_ids;
  a.in_keys = in_keys;
  a.out_adj = out_adj;
  a.out_keys = out_keys;
  a.order = GRNND_ORDER_ASCENDING;
  a.mcoef = margin_coef(c);
  a.mcoef_f32 = margin_coef_f32(c);
  a.x3 = use_x3(c) ? 1 : 0;
  a.zero16 = c.W.zero16;
  a.statp = c.W.statp;
  a.vlist_s = c.W.vlist_s;
  a.vlist_m = c.W.vlist_m;
  a.vlist_l = c.W.vlist_l;
  a.vlist_b = c.W.vlist_b;
  a.vcount = c.W.cursor + 1;
  {
    ProfScope ps(GRNND_PROF_FINAL, c.s);
    int32_t* const lists[4] = {c.W.vlist_s, c.W.vlist_m, c.W.vlist_l, c.W.vlist_b};
    HIP_OK(launch_classify(in_ids, c.lists_ready ? c.W.pool_cls : nullptr, c.order, c.n, c.R,
                           lists, c.W.cursor + 1, c.s));
    HIP_OK(launch_round(a, c.metric, true, c.compact, c.s));
  }
  return GRNND_OK;
}

// Alg. 3's schedule on a set-up context: locality order, initial pools,
// T1 x (T2 update rounds, reverse sampling unless last), output pass into
// out_adj / out_keys, or, for a batched build (out_adj null), into the spare
// pool followed by the split into the collections' rows.
int schedule(Ctx& c, uint64_t seed, int32_t* out_adj, float* out_keys) {
  int rc;
  {
    ProfScope ps(GRNND_PROF_INIT, c.s);
    HIP_OK(launch_locality_order(c.X, c.n, c.ld, seed, c.W.cell, c.W.chist, c.W.order, c.s));
    c.order = c.W.order;
  }
  int32_t *ci = c.W.pa_ids, *ni = c.W.pb_ids;
  float *ck = c.W.pa_keys, *nk = c.W.pb_keys;
  if ((rc = do_init(c, c.p.S, seed, ci, ck))) return rc;
  for (int32_t t1 = 1; t1 <= c.p.T1; ++t1) {
    for (int32_t t2 = 1; t2 <= c.p.T2; ++t2) {
      const uint32_t round = (uint32_t)((t1 - 1) * c.p.T2 + (t2 - 1));
      if ((rc = do_update(c, ci, ck, ni, nk, seed, round))) return rc;
      std::swap(ci, ni);
      std::swap(ck, nk);
    }
    if (t1 != c.p.T1) {
      if ((rc = do_reverse(c, ci, ck, ni, nk, seed, (uint32_t)t1))) return rc;
      std::swap(ci, ni);
      std::swap(ck, nk);
    }
  }
  if (out_adj) return do_final(c, ci, ck, out_adj, out_keys);
  if ((rc = do_final(c, ci, ck, ni, nk))) return rc;
  HIP_OK(launch_seg_split(ni, nk, c.n, c.R, c.seg, c.s));
  return GRNND_OK;
}

int begin(const Ctx& c) {
  HIP_OK(launch_clear(c.W.cnt, c.n, c.W.cursor, c.W.statp, c.W.zero16, c.s));
  return GRNND_OK;
}

int end(const Ctx& c, uint64_t* dev_stats) {
  if (dev_stats) HIP_OK(launch_stats_reduce(c.W.statp, dev_stats, c.s));
  return GRNND_OK;
}

}  // namespace

extern "C" {

int grnnd_version(void) { return 100; }

int grnnd_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return GRNND_OK;
}

int grnnd_profile_read(double* ms, int64_t* launches) {
  if (!ms || !launches) return fail(GRNND_EINVAL, "null output array");
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs.swap(g_prof);
  }
  for (int k = 0; k < GRNND_NPROF; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  int rc = GRNND_OK;
  for (auto& r : recs) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess && rc == GRNND_OK)
      rc = fail(GRNND_EDEVICE, "event timing failed: %s", hipGetErrorString(e));
    ms[r.kind] += t;
    launches[r.kind] += 1;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  return rc;
}

const char* grnnd_last_error(void) { return g_err.c_str(); }

int grnnd_params_default(grnnd_params* p, int32_t R, int32_t iters) {
  if (!p) return fail(GRNND_EINVAL, "params is null");
  if (R < 1 || iters < 1) return fail(GRNND_EINVAL, "R=%d, iters=%d must be >= 1", R, iters);
  *p = defaults(R, iters);
  return GRNND_OK;
}

int grnnd_workspace_size(int64_t n, int32_t d, int32_t R, const grnnd_params* p, size_t* bytes) {
  if (!bytes) return fail(GRNND_EINVAL, "bytes is null");
  if (n < 2 || d < 1 || R < 1 || R > GRNND_MAX_R)
    return fail(GRNND_EINVAL, "bad sizes n=%lld d=%d R=%d", (long long)n, d, R);
  const grnnd_params q = p ? *p : defaults(R, 1);
  if (int rc = check_params(q, R)) return rc;
  *bytes = ws_layout(nullptr, n, d, R, q).total;
  return GRNND_OK;
}

int grnnd_build_ex(const float* points, int64_t n, int32_t d, int32_t metric, int32_t R,
                   const grnnd_params* pp, uint64_t seed, int32_t* out_adj, float* out_keys,
                   uint64_t* dev_stats, void* ws, size_t ws_bytes, void* stream) {
  if (!out_adj) return fail(GRNND_EINVAL, "out_adj is null");
  Ctx c;
  int rc = setup(c, points, n, d, metric, R, pp, ws, ws_bytes, stream);
  if (rc) return rc;
  if ((rc = begin(c))) return rc;
  if ((rc = schedule(c, seed, out_adj, out_keys))) return rc;
  return end(c, dev_stats);
}

int grnnd_batch_workspace_size(const int64_t* ns, int32_t count, int32_t d, int32_t R,
                               const grnnd_params* p, size_t* bytes) {
  if (!bytes || !ns) return fail(GRNND_EINVAL, "null argument");
  if (count < 1 || count > kMaxSegs)
    return fail(GRNND_EINVAL, "count=%d out of range [1, %d]", count, kMaxSegs);
  int64_t n = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (ns[i] < 2) return fail(GRNND_EINVAL, "collection %d has n=%lld < 2", i, (long long)ns[i]);
    n += ns[i];
  }
  if (n >= (int64_t)1 << 31) return fail(GRNND_EINVAL, "%lld points in all", (long long)n);
  if (d < 1 || d > 4096 || R < 1 || R > GRNND_MAX_R)
    return fail(GRNND_EINVAL, "bad sizes d=%d R=%d", d, R);
  const grnnd_params q = p ? *p : defaults(R, 1);
  *bytes = ws_layout(nullptr, n, d, R, q, count).total;
  return GRNND_OK;
}

int grnnd_build_batch(const grnnd_batch_item* items, int32_t count, int32_t d, int32_t metric,
                      int32_t R, const grnnd_params* pp, uint64_t* dev_stats, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!items) return fail(GRNND_EINVAL, "items is null");
  if (count < 1 || count > kMaxSegs)
    return fail(GRNND_EINVAL, "count=%d out of range [1, %d]", count, kMaxSegs);
  SegTable t{};
  t.count = count;
  int64_t n = 0;
  for (int32_t i = 0; i < count; ++i) {
    const grnnd_batch_item& it = items[i];
    int rc = check_sizes(it.points, it.n, d, metric, R);
    if (rc) return fail(rc, "collection %d: %s", i, g_err.c_str());
    if (!it.out_adj) return fail(GRNND_EINVAL, "collection %d: out_adj is null", i);
    t.seg[i].base = n;
    t.seg[i].n = it.n;
    t.seg[i].seed = it.seed;
    t.seg[i].out_adj = it.out_adj;
    t.seg[i].out_keys = it.out_keys;
    n += it.n;
  }
  if (n >= (int64_t)1 << 31) return fail(GRNND_EINVAL, "%lld points in all", (long long)n);
  Ctx c;
  c.p = pp ? *pp : defaults(R, 1);
  int rc = check_params(c.p, R);
  if (rc) return rc;
  const Ws need = ws_layout(nullptr, n, d, R, c.p, count);
  if (!ws) return fail(GRNND_EINVAL, "workspace is null");
  if (ws_bytes < need.total)
    return fail(GRNND_ENOSPACE, "workspace has %zu B, needs %zu B", ws_bytes, need.total);
  if (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1))
    return fail(GRNND_EINVAL, "workspace must be 256-byte aligned");
  if ((uint64_t)n * (uint64_t)need.cap >= ((uint64_t)1 << 32))
    return fail(GRNND_ENOTSUP, "n * items per vertex exceeds 2^32");
  c.W = ws_layout(ws, n, d, R, c.p, count);
  c.n = n;
  c.d = d;
  c.metric = metric;
  c.R = R;
  c.s = static_cast<hipStream_t>(stream);
  c.d4 = (d + 3) / 4;
  c.ld = 4 * c.d4;
  c.X = c.W.xcat;
  c.seg = SegMap{c.W.vseg, c.W.segs};
  // the collections' rows, one after the other, each row zero padded to ld
  for (int32_t i = 0; i < count; ++i) {
    if (d % 4)
      HIP_OK(launch_pad_copy(items[i].points, items[i].n, d, c.W.xcat + t.seg[i].base * c.ld,
                             c.ld, c.s));
    else
      HIP_OK(hipMemcpyAsync(c.W.xcat + t.seg[i].base * c.ld, items[i].points,
                            (size_t)items[i].n * d * 4, hipMemcpyDeviceToDevice, c.s));
  }
  HIP_OK(launch_seg_fill(t, n, c.W.segs, c.W.vseg, c.s));
  if ((rc = begin(c))) return rc;
  // the output pass writes the batch's rows into the spare pool, which the
  // split hands to the collections
  if ((rc = schedule(c, items[0].seed, nullptr, nullptr))) return rc;
  return end(c, dev_stats);
}

int grnnd_build(const float* points, int64_t n, int32_t d, int32_t metric, int32_t R,
                int32_t iters, uint64_t seed, int32_t* out_adj, void* ws, size_t ws_bytes,
                void* stream) {
  if (iters < 1) return fail(GRNND_EINVAL, "iters=%d must be >= 1", iters);
  if (R < 1 || R > GRNND_MAX_R) return fail(GRNND_EINVAL, "R=%d out of range [1, 64]", R);
  const grnnd_params p = defaults(R, iters);
  return grnnd_build_ex(points, n, d, metric, R, &p, seed, out_adj, nullptr, nullptr, ws,
                        ws_bytes, stream);
}

int grnnd_init_pools(const float* points, int64_t n, int32_t d, int32_t metric, int32_t R,
                     int32_t S, uint64_t seed, int32_t* out_ids, float* out_keys,
                     uint64_t* dev_stats, void* ws, size_t ws_bytes, void* stream) {
  if (!out_ids || !out_keys) return fail(GRNND_EINVAL, "output pool is null");
  if (R < 1 || R > GRNND_MAX_R) return fail(GRNND_EINVAL, "R=%d out of range [1, 64]", R);
  grnnd_params p = defaults(R, 1);
  p.S = S;
  Ctx c;
  int rc = setup(c, points, n, d, metric, R, &p, ws, ws_bytes, stream);
  if (rc) return rc;
  if ((rc = begin(c))) return rc;
  if ((rc = do_init(c, S, seed, out_ids, out_keys))) return rc;
  return end(c, dev_stats);
}

namespace {
// The pool check of grnnd_step (params.check): one launch, then a wait for
// its verdict.
int check_pool(Ctx& c, const int32_t* ids, const float* keys) {
  static const char* const what[] = {
      "", "an id outside [-1, n)", "the row's own id", "a valid entry after padding, or padding "
      "whose key is not +inf", "an id twice", "entries not strictly ascending by (key, id)",
      "a key that is not the canonical distance"};
  HIP_OK(launch_check_pool(c.X, c.ld, c.d4, c.n, c.R, c.metric, ids, keys, c.W.check, c.s));
  unsigned long long bad = 0;
  HIP_OK(hipMemcpyAsync(&bad, c.W.check, sizeof(bad), hipMemcpyDeviceToHost, c.s));
  HIP_OK(hipStreamSynchronize(c.s));
  if (bad == ~0ull) return GRNND_OK;
  const unsigned code = (unsigned)(bad & 7u);
  return fail(GRNND_EINVAL, "read pool is not canonical: row %lld holds %s",
              (long long)(bad >> 3), code < 7 ? what[code] : "?");
}
}  // namespace

int grnnd_step(const float* points, int64_t n, int32_t d, int32_t metric, int32_t R,
               const int32_t* in_ids, const float* in_keys, int32_t* out_ids, float* out_keys,
               uint64_t seed, uint32_t round, int32_t kind, const grnnd_params* pp,
               uint64_t* dev_stats, void* ws, size_t ws_bytes, void* stream) {
  if (!in_ids || !in_keys || !out_ids || !out_keys) return fail(GRNND_EINVAL, "pool is null");
  if (in_ids == out_ids || in_keys == out_keys)
    return fail(GRNND_EINVAL, "read and write pools must not alias");
  if (kind != GRNND_STEP_UPDATE && kind != GRNND_STEP_REVERSE)
    return fail(GRNND_EINVAL, "kind=%d unknown", kind);
  Ctx c;
  int rc = setup(c, points, n, d, metric, R, pp, ws, ws_bytes, stream);
  if (rc) return rc;
  if (c.p.check && (rc = check_pool(c, in_ids, in_keys))) return rc;
  if ((rc = begin(c))) return rc;
  if (kind == GRNND_STEP_UPDATE)
    rc = do_update(c, in_ids, in_keys, out_ids, out_keys, seed, round);
  else
    rc = do_reverse(c, in_ids, in_keys, out_ids, out_keys, seed, round);
  if (rc) return rc;
  return end(c, dev_stats);
}

int grnnd_finalize(const float* points, int64_t n, int32_t d, int32_t metric, int32_t R,
                   const int32_t* in_ids, const float* in_keys, int32_t* out_adj,
                   float* out_keys, uint64_t* dev_stats, void* ws, size_t ws_bytes,
                   void* stream) {
  if (!in_ids || !in_keys || !out_adj) return fail(GRNND_EINVAL, "pool is null");
  Ctx c;
  int rc = setup(c, points, n, d, metric, R, nullptr, ws, ws_bytes, stream);
  if (rc) return rc;
  if ((rc = begin(c))) return rc;
  if ((rc = do_final(c, in_ids, in_keys, out_adj, out_keys))) return rc;
  return end(c, dev_stats);
}

int grnnd_tile_probe(const float* points, int64_t n, int32_t d, int32_t metric, int32_t R,
                     const grnnd_params* p, const int32_t* ids, int64_t nv, float* out_tile,
                     float* out_band, float* out_canon, void* ws, size_t ws_bytes, void* stream) {
  if (!ids || !out_tile || !out_band || !out_canon) return fail(GRNND_EINVAL, "argument is null");
  if (nv < 0 || nv >= ((int64_t)1 << 31)) return fail(GRNND_EINVAL, "nv=%lld out of range", (long long)nv);
  Ctx c;
  int rc = setup(c, points, n, d, metric, R, p, ws, ws_bytes, stream);
  if (rc) return rc;
  if (nv == 0) return GRNND_OK;
  if ((rc = ensure_narrow(c))) return rc;
  if ((rc = ensure_rexact(c))) return rc;
  RoundArgs a{};
  set_narrow(c, a);
  a.X = c.X;
  a.n = c.n;
  a.d = c.d;
  a.d4 = c.d4;
  a.ld = c.ld;
  a.R = c.R;
  a.mcoef = margin_coef(c);
  a.mcoef_f32 = margin_coef_f32(c);
  a.x3 = use_x3(c) ? 1 : 0;
  HIP_OK(launch_tile_probe(a, c.metric, ids, nv, out_tile, out_band, out_canon, c.s));
  return GRNND_OK;
}

namespace {
// Search workspace: a 256-byte zero block, the medoid's scratch and its
// result, then (d % 4 != 0) row-padded copies of the points and queries.
struct SearchWs {
  size_t medoid_off, entry_off, xp_off, qp_off, total;
};
SearchWs search_ws(int64_t n, int32_t d, int64_t nq) {
  SearchWs w;
  w.medoid_off = 256;
  w.entry_off = w.medoid_off + align_up(medoid_layout(n, d).total);
  w.xp_off = w.entry_off + 256;
  w.qp_off = w.xp_off;
  w.total = w.xp_off;
  if (d % 4) {
    w.qp_off = w.xp_off + align_up((size_t)n * round_up(d, 4) * 4);
    w.total = w.qp_off + align_up((size_t)nq * round_up(d, 4) * 4);
  }
  return w;
}
}  // namespace

int grnnd_search_workspace_size(int64_t n, int32_t d, int64_t nq, size_t* bytes) {
  if (!bytes) return fail(GRNND_EINVAL, "bytes is null");
  if (n < 1 || d < 1 || nq < 0) return fail(GRNND_EINVAL, "bad sizes");
  *bytes = search_ws(n, d, nq).total;
  return GRNND_OK;
}

int grnnd_medoid(const float* points, int64_t n, int32_t d, int64_t* out_entry, void* ws,
                 size_t ws_bytes, void* stream) {
  if (!points || !out_entry) return fail(GRNND_EINVAL, "null pointer argument");
  if (n < 1 || n >= (int64_t)1 << 31) return fail(GRNND_EINVAL, "n out of range");
  if (d < 1 || d > 4096) return fail(GRNND_EINVAL, "d out of range");
  const SearchWs w = search_ws(n, d, 0);
  if (!ws) return fail(GRNND_EINVAL, "workspace is null");
  if (ws_bytes < w.entry_off)
    return fail(GRNND_ENOSPACE, "workspace has %zu B, needs %zu B", ws_bytes, w.entry_off);
  if (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1))
    return fail(GRNND_EINVAL, "workspace must be 256-byte aligned");
  HIP_OK(launch_medoid(points, n, d, static_cast<char*>(ws) + w.medoid_off, out_entry,
                       static_cast<hipStream_t>(stream)));
  return GRNND_OK;
}

int grnnd_search(const float* points, int64_t n, int32_t d, int32_t metric, const int32_t* adj,
                 int32_t R, int64_t entry, const float* queries, int64_t nq, int32_t k,
                 int32_t L, int32_t* out_ids, float* out_keys, void* ws, size_t ws_bytes,
                 void* stream) {
  if (!points || !adj || !queries || !out_ids || !out_keys)
    return fail(GRNND_EINVAL, "null pointer argument");
  if (n < 1 || n >= (int64_t)1 << 31) return fail(GRNND_EINVAL, "n out of range");
  if (d < 1 || d > 4096) return fail(GRNND_EINVAL, "d out of range");
  if (metric != 0 && metric != 1) return fail(GRNND_EINVAL, "metric unknown");
  if (R < 1 || R > GRNND_MAX_R) return fail(GRNND_EINVAL, "R out of range");
  if (k < 1 || L < k || L > 256) return fail(GRNND_EINVAL, "need 1 <= k <= L <= 256");
  if (entry >= n) return fail(GRNND_EINVAL, "entry out of range");
  if (nq < 0 || nq >= (int64_t)1 << 31) return fail(GRNND_EINVAL, "nq out of range");
  if (nq == 0) return GRNND_OK;
  const SearchWs w = search_ws(n, d, nq);
  if (!ws) return fail(GRNND_EINVAL, "workspace is null");
  if (ws_bytes < w.total) return fail(GRNND_ENOSPACE, "workspace has %zu B, needs %zu B", ws_bytes, w.total);
  if (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1))
    return fail(GRNND_EINVAL, "workspace must be 256-byte aligned");
  if (d % 4 == 0 && ((reinterpret_cast<uintptr_t>(points) | reinterpret_cast<uintptr_t>(queries)) & 15))
    return fail(GRNND_EINVAL, "points and queries must be 16-byte aligned");
  const size_t lds = search_lds_bytes(R, round_up(d, 4));
  if (lds > max_lds_bytes()) return fail(GRNND_ENOTSUP, "R, d too large for the search kernel");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* wb = static_cast<char*>(ws);
  SearchArgs a{};
  a.n = n;
  a.d = d;
  a.d4 = (d + 3) / 4;
  a.metric = metric;
  a.adj = adj;
  a.R = R;
  a.entry = entry;
  a.entry_dev = nullptr;
  a.nq = nq;
  a.k = k;
  a.L = L;
  a.out_ids = out_ids;
  a.out_keys = out_keys;
  float* zero = reinterpret_cast<float*>(wb);  // first 256 bytes: zero block
  a.zero16 = zero;
  HIP_OK(launch_clear(nullptr, 0, nullptr, nullptr, zero, s));
  if (entry < 0) {  // the default entry: the approximate medoid (Section 4.1)
    int64_t* e = reinterpret_cast<int64_t*>(wb + w.entry_off);
    HIP_OK(launch_medoid(points, n, d, wb + w.medoid_off, e, s));
    a.entry_dev = e;
  }
  if (d % 4) {
    float* xp = reinterpret_cast<float*>(wb + w.xp_off);
    float* qp = reinterpret_cast<float*>(wb + w.qp_off);
    HIP_OK(launch_pad_copy(points, n, d, xp, 4 * a.d4, s));
    HIP_OK(launch_pad_copy(queries, nq, d, qp, 4 * a.d4, s));
    a.X = xp;
    a.Q = qp;
    a.ld = a.ldq = 4 * a.d4;
  } else {
    a.X = points;
    a.Q = queries;
    a.ld = a.ldq = d;
  }
  {
    ProfScope ps(GRNND_PROF_SEARCH, s);
    HIP_OK(launch_search(a, s));
  }
  return GRNND_OK;
}

}  // extern "C"
