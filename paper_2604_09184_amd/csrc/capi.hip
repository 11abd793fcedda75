// C-ABI of the library (declared in include/nbody.h): argument validation, context workspace,
// launch planning and the orchestration of kick / jump / drift / encounter kernels on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <functional>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/nbody.h"

#include "internal.hpp"

using namespace nbk;

// Workspace of nbody_kick_noalloc (see scratch_ptr below): 32 MiB per device.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};

enum BufId { B_PART, B_PART_CE, B_CNT, B_ROWBUF, B_ROWTOT, B_BSUM, B_ROWSUM, B_ROWMASK, B_MOM_A, B_MOM_B, B_THR, B_EPARTS,
             B_ADJ_STATES, B_XA, B_VA, B_LSUM, B_B_OFFS, B_B_ORDER,
             B_B_CFG, B_B_THR, B_B_QUEUE, B_T_XM, B_T_V, B_B_PART, B_PERM, B_CELL,
             B_RANGE, B_CCOUNT, B_CCURSOR, B_MPART, B_UNI, B_VKEY, B_GIN, B_GSIZE,
             B_GSTART, B_GFILL, B_GMEM, B_GROOT, B_GCNT, B_HPAIRS, B_HCOUNT, B_HLAB, B_LTHR, B_ADEG, B_AOFF,
             B_AFILL, B_ADJ, B_LSKIP, B_ATOT, B_ETHR, B_GSIZE2, B_GCNT2, B_GSLICE, B_ALONG, B_NUM };

}  // namespace

struct nbody_ctx {
  nbody_params p{};
  std::string err;
  Buf buf[B_NUM];
  int R = 64;               // partner slots per (row, j-chunk) in the emission buffer (at most)
  int locality_min_n = 4096;  // lane permutation by position for n at least this
  int locality_every = 10;    // steps between refreshes of the lane permutation in nbody_step
  int target_waves = 32768; // pair-kernel waves per launch: 32 per SIMD, for load balance
  // batched tile per size class: 1 = one wave per system (systems of at most 256 bodies),
  // 0 = one workgroup per system
  int32_t tiles[nbk::kBuckets] = {0, 0, 0, 0, 0, 0};
  bool tuned = false;
  std::map<int64_t, int32_t> step_path;   // n -> path chosen by nbody_autotune_step
  std::vector<int64_t> h_offs;   // host staging kept alive across asynchronous copies
  std::vector<int32_t> h_order;
};

namespace {

int fail(nbody_ctx *c, int code, const char *fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  if (c) c->err = msg;
  return code;
}

int hip_fail(nbody_ctx *c, hipError_t e, const char *where) {
  return fail(c, NBODY_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIPCHK(c, expr, where)                         \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(c, e_, where); \
  } while (0)

void *ensure(nbody_ctx *c, BufId id, size_t bytes) {
  Buf &b = c->buf[id];
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return b.p;
  if (b.p) {
    (void)hipDeviceSynchronize();
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    b.p = nullptr;
    return nullptr;
  }
  b.bytes = bytes;
  return b.p;
}

// ensure() for a buffer that must be zero when first handed out (hipMemset on (re)allocation;
// its users leave it zero after every use).
void *ensure_zeroed(nbody_ctx *c, BufId id, size_t bytes) {
  Buf &b = c->buf[id];
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return b.p;
  void *p = ensure(c, id, bytes);
  if (p && hipMemset(p, 0, bytes) != hipSuccess) return nullptr;
  return p;
}

bool params_ok(const nbody_params *p) {
  return p && p->m0 > 0 && p->n1 >= 0 && p->n2 >= 0 && p->f_in >= 0 && p->f_in < 1 &&
         (p->precision == NBODY_PREC_F64 || p->precision == NBODY_PREC_SPLIT) && p->G == p->G &&
         p->dt == p->dt;
}

// Device pointer, aligned to 32 bytes.
int check_dev(nbody_ctx *c, const void *ptr, const char *name, bool required) {
  if (!ptr) return required ? fail(c, NBODY_E_INVAL, "%s is NULL", name) : NBODY_OK;
  if ((uintptr_t)ptr & 31u) return fail(c, NBODY_E_INVAL, "%s is not 32-byte aligned", name);
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, NBODY_E_INVAL, "%s is not a HIP allocation", name);
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
    return fail(c, NBODY_E_INVAL, "%s is not device memory", name);
  return NBODY_OK;
}

int check_n(nbody_ctx *c, int64_t n) {
  if (!c) return NBODY_E_INVAL;
  if (n <= 0 || n > (int64_t)1 << 28) return fail(c, NBODY_E_INVAL, "n = %lld out of range", (long long)n);
  return NBODY_OK;
}

#define TRY(expr)               \
  do {                          \
    int r_ = (expr);            \
    if (r_ != NBODY_OK) return r_; \
  } while (0)

// j-chunking: enough waves to fill the chip, chunks of at least 64 bodies, or 32 for systems of
// at most 4096 bodies, twice the waves of a launch that otherwise runs one wave per SIMD
// (measured: 2048-body step 25.0 -> 21.8 us). The chunking depends on n alone, so a launch with
// the encounter list sums in the same order as one without.
void plan(const nbody_ctx *c, int n, int &S, int &chunk) {
  const int iwaves = (n + 63) / 64;
  int s = (c->target_waves + iwaves - 1) / iwaves;
  const int minchunk = n <= 4096 ? 32 : 64;
  const int smax = (n + minchunk - 1) / minchunk;
  if (s > smax) s = smax;
  if (s < 1) s = 1;
  chunk = (n + s - 1) / s;
  S = (n + chunk - 1) / chunk;
}

// Lane permutation grouping spatially close bodies into waves (no effect on any result bit);
// null below the size where it pays.
// Workspace of the lane permutation for n bodies (the cell counters start at zero; the kernels
// leave them at zero after every use).
int locality_bufs(nbody_ctx *c, int n, hipStream_t st) {
  const int nb = nblocks(n);
  const bool fresh = c->buf[B_CCOUNT].p == nullptr;
  if (!ensure(c, B_PERM, (size_t)n * sizeof(int)) ||
      !ensure(c, B_CELL, (size_t)n * sizeof(unsigned short)) ||
      !ensure(c, B_RANGE, (size_t)nb * sizeof(float2)) ||
      !ensure(c, B_CCOUNT, (size_t)locality_cells() * sizeof(unsigned)) ||
      !ensure(c, B_CCURSOR, (size_t)locality_cells() * sizeof(unsigned)))
    return fail(c, NBODY_E_NOMEM, "workspace allocation failed (locality)");
  if (fresh)
    HIPCHK(c, hipMemsetAsync(c->buf[B_CCOUNT].p, 0, (size_t)locality_cells() * sizeof(unsigned), st), "memset");
  return NBODY_OK;
}

int locality(nbody_ctx *c, int n, const double4 *xm, hipStream_t st, const int **perm) {
  *perm = nullptr;
  if (n < c->locality_min_n) return NBODY_OK;
  TRY(locality_bufs(c, n, st));
  int *p = (int *)c->buf[B_PERM].p;
  HIPCHK(c, launch_locality(xm, n, (float2 *)c->buf[B_RANGE].p, (unsigned short *)c->buf[B_CELL].p,
                            (unsigned *)c->buf[B_CCOUNT].p, (unsigned *)c->buf[B_CCURSOR].p, p, st),
         "locality");
  *perm = p;
  return NBODY_OK;
}

// Device flag {1, m} when all masses equal m (computed once per call; masses never change).
int mass_check(nbody_ctx *c, int n, const double4 *xm, hipStream_t st, const double2 **uni) {
  double2 *part = (double2 *)ensure(c, B_MPART, (size_t)nblocks(n) * sizeof(double2));
  double2 *u = (double2 *)ensure(c, B_UNI, sizeof(double2));
  if (!part || !u) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (mass check)");
  HIPCHK(c, launch_mass_check(xm, n, part, u, st), "mass check");
  *uni = u;
  return NBODY_OK;
}

int make_kick_args(nbody_ctx *c, int n, const double *xm, const double *thr, bool need_force,
                   bool need_ce, bool need_emit, KickArgs &a) {
  plan(c, n, a.nchunk, a.chunk);
  a.perm = nullptr;
  a.uni = nullptr;
  a.xm = reinterpret_cast<const double4 *>(xm);
  a.thr = reinterpret_cast<const double4 *>(thr);
  a.n = n;
  a.f_in = c->p.f_in;
  // partner slots per (row, chunk): a row-chunk that overflows is rescanned at O(chunk) cost
  a.R = std::min(c->R, std::max(16, a.chunk / 32));
  const size_t sn = (size_t)a.nchunk * n;
  a.part = need_force ? (double4 *)ensure(c, B_PART, sn * sizeof(double4)) : nullptr;
  a.part_ce = need_ce ? (double4 *)ensure(c, B_PART_CE, sn * sizeof(double4)) : nullptr;
  a.cnt = need_emit ? (int *)ensure(c, B_CNT, sn * sizeof(int)) : nullptr;
  a.rowbuf = need_emit ? (int *)ensure(c, B_ROWBUF, sn * (size_t)a.R * sizeof(int)) : nullptr;
  if ((need_force && !a.part) || (need_ce && !a.part_ce) || (need_emit && (!a.cnt || !a.rowbuf)))
    return fail(c, NBODY_E_NOMEM, "workspace allocation failed (n = %d, chunks = %d)", n, a.nchunk);
  // per-row totals and chunk masks for the emission (zero between uses: set by the pair kernel,
  // cleared by the emission that follows it)
  a.rowsum = nullptr;
  a.rowmask = nullptr;
  if (need_emit && a.nchunk <= 64 * kRowMaskWords) {
    a.rowsum = (int *)ensure_zeroed(c, B_ROWSUM, (size_t)n * sizeof(int));
    a.rowmask = (unsigned long long *)ensure_zeroed(c, B_ROWMASK,
                                                     (size_t)n * kRowMaskWords * sizeof(unsigned long long));
    if (!a.rowsum || !a.rowmask) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (row masks)");
  }
  return NBODY_OK;
}

int emit_list(nbody_ctx *c, const KickArgs &a, int32_t *pairs, int64_t cap, int64_t *count,
              hipStream_t st, unsigned long long *overflow = nullptr) {
  const int nb = nblocks(a.n);
  int64_t *rowtot = (int64_t *)ensure(c, B_ROWTOT, (size_t)a.n * sizeof(int64_t));
  int64_t *bsum = (int64_t *)ensure(c, B_BSUM, (size_t)nb * sizeof(int64_t));
  if (!rowtot || !bsum) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (emission)");
  HIPCHK(c, launch_emit(a, pairs, cap, count, rowtot, bsum, st, overflow), "encounter emission");
  return NBODY_OK;
}

// lam += VJP of the kick v' = v + h a(x) at positions xm (adds to lam_x, including dL/dm).
// uni: the equal-mass flag of xm (from mass_check; masses never change along a trajectory).
// perm: a lane permutation to reuse (any permutation gives the same bits), or null to build one
// for xm.
int kick_vjp(nbody_ctx *c, int n, const double4 *xm, const double4 *thr, const double2 *uni,
             const double4 *lam_v, double h, double4 *lam_x, hipStream_t st, int napply = 1,
             const int *perm = nullptr) {
  KickArgs a;
  TRY(make_kick_args(c, n, (const double *)xm, (const double *)thr, true, false, false, a));
  if (perm) a.perm = perm;
  else TRY(locality(c, n, xm, st, &a.perm));
  HIPCHK(c, launch_kick_vjp(xm, thr, a.perm, uni, lam_v, h, c->p.G, c->p.f_in, n, a.nchunk, a.chunk, napply,
                            a.part, lam_x, st), "kick vjp");
  return NBODY_OK;
}

int jump_vjp(nbody_ctx *c, int n, const double4 *xm, const double4 *v, double h, double4 *lam_x,
             double4 *lam_v, hipStream_t st) {
  double4 *parts = (double4 *)ensure(c, B_LSUM, (size_t)nblocks(n) * sizeof(double4));
  if (!parts) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (adjoint)");
  HIPCHK(c, launch_jump_vjp(xm, v, h, c->p.m0, n, parts, lam_x, lam_v, st), "jump vjp");
  return NBODY_OK;
}

// ------------------------------------------------------------------ batched ensembles
int size_class_host(int64_t n) {
  int b = 0;
  while (b < kBuckets - 1 && n > (int64_t(64) << b)) ++b;
  return b;
}

int check_offs(nbody_ctx *c, int32_t nsys, const int64_t *offs) {
  if (nsys <= 0 || !offs) return fail(c, NBODY_E_INVAL, "nsys <= 0 or offs NULL");
  if (offs[0] != 0) return fail(c, NBODY_E_INVAL, "offs[0] must be 0");
  for (int32_t s = 0; s < nsys; ++s) {
    const int64_t n = offs[s + 1] - offs[s];
    if (n < 1 || n > batched_max_group_n())
      return fail(c, NBODY_E_INVAL, "system %d has %lld bodies (1..%d supported)", s, (long long)n,
                  batched_max_group_n());
  }
  return NBODY_OK;
}

int grid_size(nbody_ctx *c, int *grid) {
  int dev = 0, per = 0;
  hipDeviceProp_t prop;
  HIPCHK(c, hipGetDevice(&dev), "device");
  HIPCHK(c, hipGetDeviceProperties(&prop, dev), "device properties");
  HIPCHK(c, batched_occupancy(&per), "occupancy");
  if (per < 1) per = 1;
  *grid = prop.multiProcessorCount * per;
  return NBODY_OK;
}

// Launches the persistent kernel over the systems laid out by host offsets h_offs with the tile
// table `tiles` (host, kBuckets codes).
// only_class >= 0: run only the systems of that size class (the others are left untouched).
int run_batched(nbody_ctx *c, int32_t nsys, const int32_t *tiles, double4 *xm, double4 *v, int32_t nsteps,
                unsigned long long *npairs, hipStream_t st, int only_class = -1) {
  std::vector<int64_t> &h_offs = c->h_offs;
  std::vector<int32_t> &h_order = c->h_order;
  const int64_t total = h_offs[nsys];
  BatchLaunch b;
  TRY(grid_size(c, &b.grid));
  int64_t *d_offs = (int64_t *)ensure(c, B_B_OFFS, (size_t)(nsys + 1) * sizeof(int64_t));
  int32_t *d_order = (int32_t *)ensure(c, B_B_ORDER, (size_t)nsys * sizeof(int32_t));
  int32_t *d_cfg = (int32_t *)ensure(c, B_B_CFG, kBuckets * sizeof(int32_t));
  double4 *d_thr = (double4 *)ensure(c, B_B_THR, (size_t)total * sizeof(double4));
  double4 *d_part = (double4 *)ensure(c, B_B_PART, (size_t)b.grid * 2 * kBatchedWaves * 2 * 64 * sizeof(double4));
  unsigned *d_q = (unsigned *)ensure(c, B_B_QUEUE, 256);
  if (!d_offs || !d_order || !d_cfg || !d_thr || !d_part || !d_q)
    return fail(c, NBODY_E_NOMEM, "workspace allocation failed (batched)");
  h_order.clear();
  for (int32_t s = 0; s < nsys; ++s)
    if (only_class < 0 || size_class_host(h_offs[s + 1] - h_offs[s]) == only_class) h_order.push_back(s);
  std::stable_sort(h_order.begin(), h_order.end(), [&](int32_t a, int32_t b) {
    return h_offs[a + 1] - h_offs[a] > h_offs[b + 1] - h_offs[b];
  });
  const int32_t nrun = (int32_t)h_order.size();
  HIPCHK(c, hipMemcpyAsync(d_offs, h_offs.data(), (nsys + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st), "copy");
  if (nrun > 0)
    HIPCHK(c, hipMemcpyAsync(d_order, h_order.data(), nrun * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy");
  HIPCHK(c, hipMemcpyAsync(d_cfg, tiles, kBuckets * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy");
  b.offs = d_offs; b.order = d_order; b.cfg = d_cfg; b.nsys = nrun; b.nsteps = nsteps;
  b.xm = xm; b.v = v; b.thr = d_thr; b.part = d_part; b.npairs = npairs; b.queue = d_q;
  const nbody_params &p = c->p;
  b.G = p.G; b.m0 = p.m0; b.dt = p.dt; b.f_in = p.f_in;
  b.cH = ((p.n1 * p.n1 * p.n1) * (p.n1 * p.n1 * p.n1)) / 9.0;
  b.n2dt = p.n2 * p.dt;
  b.cV = b.n2dt * b.n2dt;
  b.n1 = p.n1;
  HIPCHK(c, launch_batched(b, st), "batched launch");
  // the host staging vectors (and the tile table) must outlive the copies above
  HIPCHK(c, hipStreamSynchronize(st), "batched sync");
  return NBODY_OK;
}

// ------------------------------------------------------------------ close-encounter drift
constexpr double kCeTol = 1e-14;   // Bulirsch-Stoer tolerance, relative to the group's scales

struct GroupBufs {
  int *in, *gsize, *gstart, *gfill, *gmem, *groot, *counter;
};

int group_bufs(nbody_ctx *c, int n, GroupBufs &g) {
  const size_t b = (size_t)n * sizeof(int);
  g.in = (int *)ensure(c, B_GIN, b);
  g.gsize = (int *)ensure(c, B_GSIZE, b);
  g.gstart = (int *)ensure(c, B_GSTART, b);
  g.gfill = (int *)ensure(c, B_GFILL, b);
  g.gmem = (int *)ensure(c, B_GMEM, b);
  g.groot = (int *)ensure(c, B_GROOT, b);
  g.counter = (int *)ensure(c, B_GCNT, kGroupCounters * sizeof(int));
  if (!g.in || !g.gsize || !g.gstart || !g.gfill || !g.gmem || !g.groot || !g.counter)
    return fail(c, NBODY_E_NOMEM, "workspace allocation failed (groups)");
  return NBODY_OK;
}

// Checks the collision arguments and fills the kernel's view of them (radius null: no collisions).
int collide_args(nbody_ctx *c, int n, const nbody_collisions *col, CeCollide &cc) {
  cc = CeCollide{nullptr, 0.0, nullptr, nullptr, 0, nullptr, 0, n};
  if (!col) return NBODY_OK;
  TRY(check_dev(c, col->radius, "col->radius", true));
  TRY(check_dev(c, col->count, "col->count", true));
  if (!(col->f >= 0.0) || !std::isfinite(col->f)) return fail(c, NBODY_E_INVAL, "col->f must be finite and >= 0");
  if (col->cap < 0) return fail(c, NBODY_E_INVAL, "col->cap < 0");
  if (col->cap > 0) {
    TRY(check_dev(c, col->merges, "col->merges", true));
    TRY(check_dev(c, col->time, "col->time", true));
  }
  cc.radius = col->radius;
  cc.f = col->f;
  cc.merges = col->merges;
  cc.mtime = col->time;
  cc.cap = col->cap;
  cc.count = (unsigned long long *)col->count;
  return NBODY_OK;
}

// Member lists of the groups given by labels; then the close-encounter integration of every group
// over h (the other bodies are not touched here).
int ce_drift(nbody_ctx *c, int n, double4 *xm, double4 *v, const double4 *thr, const int *labels,
             const GroupBufs &g, double h, unsigned long long *stats, const CeCollide &col, hipStream_t st) {
  HIPCHK(c, launch_group_lists(labels, n, g.in, g.gsize, g.gstart, g.gfill, g.gmem, g.groot, g.counter,
                               false, st), "group lists");
  const nbody_params &p = c->p;
  LevelThr lt{};
  lt.thr[0] = thr;
  lt.nl = 1;
  HIPCHK(c, launch_ce_drift(xm, v, thr, g.gmem, g.gstart, g.gsize, g.groot, g.counter, n / 2 + 1, p.G, p.m0,
                            p.f_in, h, kCeTol, stats, col, lt, st), "close-encounter drift");
  return NBODY_OK;
}

// ------------------------------------------------------------------ allocation-free kick
// Workspace of nbody_kick_noalloc: a file-scope device array, one copy per device, held until the
// process ends. Host code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): it uses the device address that hipGetSymbolAddress returns, looked up
// once per device on the first call made with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first call on the device).
int scratch_ptr(nbody_ctx *c, void **out) {
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev), "device");
  if (dev < 0 || dev >= kMaxDevices) return fail(c, NBODY_E_INVAL, "device %d beyond the supported %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    HIPCHK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch address");
    if (!ptr) return fail(c, NBODY_E_HIP, "scratch address: null");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return NBODY_OK;
}

}  // namespace

extern "C" {

const char *nbody_version(void) { return "nbody-mi355x 0.1 (gfx950, binary64 vector ALU)"; }

int nbody_create(nbody_ctx **out, const nbody_params *p) {
  if (!out) return NBODY_E_INVAL;
  *out = nullptr;
  if (!params_ok(p)) return NBODY_E_INVAL;
  nbody_ctx *c = new (std::nothrow) nbody_ctx();
  if (!c) return NBODY_E_NOMEM;
  c->p = *p;
  *out = c;
  return NBODY_OK;
}

int nbody_destroy(nbody_ctx *c) {
  if (!c) return NBODY_E_INVAL;
  (void)hipDeviceSynchronize();
  for (auto &b : c->buf)
    if (b.p) (void)hipFree(b.p);
  delete c;
  return NBODY_OK;
}

int nbody_set_params(nbody_ctx *c, const nbody_params *p) {
  if (!c) return NBODY_E_INVAL;
  if (!params_ok(p)) return fail(c, NBODY_E_INVAL, "invalid parameters");
  c->p = *p;
  c->step_path.clear();   // choices of the small-N switch were timed with the old parameters
  return NBODY_OK;
}

const char *nbody_last_error(const nbody_ctx *c) { return c ? c->err.c_str() : "null context"; }

int nbody_reserve(nbody_ctx *c, int64_t n, uint32_t what, void *stream) {
  TRY(check_n(c, n));
  if (what & ~(uint32_t)(NBODY_RESERVE_KICK | NBODY_RESERVE_LIST | NBODY_RESERVE_CE))
    return fail(c, NBODY_E_INVAL, "unknown reservation flags 0x%x", what);
  hipStream_t st = (hipStream_t)stream;
  const int N = (int)n;
  KickArgs a;
  TRY(make_kick_args(c, N, nullptr, nullptr, (what & NBODY_RESERVE_KICK) != 0, (what & NBODY_RESERVE_CE) != 0,
                     (what & NBODY_RESERVE_LIST) != 0, a));
  if ((what & NBODY_RESERVE_LIST) &&
      (!ensure(c, B_ROWTOT, (size_t)n * sizeof(int64_t)) || !ensure(c, B_BSUM, (size_t)nblocks(n) * sizeof(int64_t))))
    return fail(c, NBODY_E_NOMEM, "workspace allocation failed (emission)");
  const int nbf = fin_blocks(n);
  if (!ensure(c, B_THR, (size_t)n * sizeof(double4)) || !ensure(c, B_MOM_A, (size_t)nbf * sizeof(double4)) ||
      !ensure(c, B_MOM_B, (size_t)nbf * sizeof(double4)) ||
      !ensure(c, B_MPART, (size_t)nblocks(n) * sizeof(double2)) || !ensure(c, B_UNI, sizeof(double2)))
    return fail(c, NBODY_E_NOMEM, "workspace allocation failed (step)");
  if (N >= c->locality_min_n) TRY(locality_bufs(c, N, st));
  HIPCHK(c, hipStreamSynchronize(st), "reserve sync");
  return NBODY_OK;
}

int nbody_rcrit(nbody_ctx *c, int64_t n, const double *xm, const double *v, double *thr,
                void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  TRY(check_dev(c, thr, "thr", true));
  const nbody_params &p = c->p;
  const double cH = ((p.n1 * p.n1 * p.n1) * (p.n1 * p.n1 * p.n1)) / 9.0;
  const double t = p.n2 * p.dt;
  const double cV = t * t;
  HIPCHK(c, launch_rcrit((const double4 *)xm, (const double4 *)v, (double4 *)thr, (int)n, p.m0, cH, cV,
                         p.n1, t, (hipStream_t)stream), "rcrit");
  return NBODY_OK;
}

int nbody_kick(nbody_ctx *c, int64_t n, const double *xm, const double *thr, double *v, double h,
               double *acc, double *acc_ce, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, thr, "thr", true));
  TRY(check_dev(c, v, "v", false));
  TRY(check_dev(c, acc, "acc", false));
  TRY(check_dev(c, acc_ce, "acc_ce", false));
  KickArgs a;
  TRY(make_kick_args(c, (int)n, xm, thr, true, acc_ce != nullptr, false, a));
  hipStream_t st = (hipStream_t)stream;
  TRY(locality(c, (int)n, a.xm, st, &a.perm));
  TRY(mass_check(c, (int)n, a.xm, st, &a.uni));
  HIPCHK(c, launch_pairs(a, true, false, acc_ce != nullptr, c->p.precision == NBODY_PREC_SPLIT, st),
         "kick pairs");
  HIPCHK(c, launch_finalize(a.part, a.part_ce, a.nchunk, (int)n, c->p.G, h, 1, a.xm, (double4 *)v,
                            (double4 *)acc, (double4 *)acc_ce, nullptr, st), "kick finalize");
  return NBODY_OK;
}

int nbody_kick_noalloc(nbody_ctx *c, int64_t n, const double *xm, const double *thr, double *v,
                       double h, double *acc, double *acc_ce, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, thr, "thr", true));
  TRY(check_dev(c, v, "v", false));
  TRY(check_dev(c, acc, "acc", false));
  TRY(check_dev(c, acc_ce, "acc_ce", false));
  void *base = nullptr;
  TRY(scratch_ptr(c, &base));
  const int N = (int)n;
  const bool ce = acc_ce != nullptr;
  // layout: mass-check partials, the equal-mass flag, then the [S][n] partial sums (and their
  // close-encounter parts), each 256-byte aligned; S is the usual plan, lowered until it fits
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t b_mpart = up((size_t)nblocks(N) * sizeof(double2));
  const size_t b_uni = up(sizeof(double2));
  const size_t per_chunk = up((size_t)N * sizeof(double4)) * (ce ? 2 : 1);
  if (b_mpart + b_uni + per_chunk > kScratchBytes)
    return fail(c, NBODY_E_INVAL, "n = %lld needs %zu bytes of workspace, beyond the %zu of nbody_kick_noalloc",
                (long long)n, b_mpart + b_uni + per_chunk, kScratchBytes);
  KickArgs a;
  plan(c, N, a.nchunk, a.chunk);
  const int smax = (int)std::min<size_t>((kScratchBytes - b_mpart - b_uni) / per_chunk, (size_t)INT32_MAX);
  if (a.nchunk > smax) {
    a.chunk = (N + smax - 1) / smax;
    a.nchunk = (N + a.chunk - 1) / a.chunk;
  }
  unsigned char *p = (unsigned char *)base;
  double2 *mpart = (double2 *)p;
  double2 *uni = (double2 *)(p + b_mpart);
  unsigned char *q = p + b_mpart + b_uni;
  a.part = (double4 *)q;
  a.part_ce = ce ? (double4 *)(q + up((size_t)a.nchunk * N * sizeof(double4))) : nullptr;
  a.xm = reinterpret_cast<const double4 *>(xm);
  a.thr = reinterpret_cast<const double4 *>(thr);
  a.perm = nullptr;   // identity lanes: every body's sum has the same bits under any lane order
  a.uni = uni;
  a.n = N;
  a.f_in = c->p.f_in;
  a.cnt = nullptr;
  a.rowbuf = nullptr;
  a.R = 0;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(c, launch_mass_check(a.xm, N, mpart, uni, st), "mass check");
  HIPCHK(c, launch_pairs(a, true, false, ce, c->p.precision == NBODY_PREC_SPLIT, st), "kick pairs");
  HIPCHK(c, launch_finalize(a.part, a.part_ce, a.nchunk, N, c->p.G, h, 1, a.xm, (double4 *)v,
                            (double4 *)acc, (double4 *)acc_ce, nullptr, st), "kick finalize");
  return NBODY_OK;
}

int nbody_encounters(nbody_ctx *c, int64_t n, const double *xm, const double *thr, int32_t *pairs,
                     int64_t cap, int64_t *count, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, thr, "thr", true));
  TRY(check_dev(c, count, "count", true));
  if (cap < 0) return fail(c, NBODY_E_INVAL, "cap < 0");
  if (cap > 0) TRY(check_dev(c, pairs, "pairs", true));
  KickArgs a;
  TRY(make_kick_args(c, (int)n, xm, thr, false, false, true, a));
  hipStream_t st = (hipStream_t)stream;
  TRY(locality(c, (int)n, a.xm, st, &a.perm));
  HIPCHK(c, launch_pairs(a, false, true, false, false, st), "encounter pairs");
  return emit_list(c, a, pairs, cap, count, st);
}

int nbody_jump(nbody_ctx *c, int64_t n, double *xm, const double *v, double h, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  const int nb = fin_blocks(n);
  double4 *mom = (double4 *)ensure(c, B_MOM_A, (size_t)nb * sizeof(double4));
  if (!mom) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (momentum)");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(c, launch_momentum((const double4 *)xm, (const double4 *)v, (int)n, mom, st), "momentum");
  HIPCHK(c, launch_jump((double4 *)xm, mom, nb, (int)n, h, c->p.m0, st), "jump");
  return NBODY_OK;
}

int nbody_drift(nbody_ctx *c, int64_t n, double *xm, double *v, double h, uint32_t *status,
                void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  TRY(check_dev(c, status, "status", false));
  HIPCHK(c, launch_drift((double4 *)xm, (double4 *)v, (int)n, h, c->p.G * c->p.m0, status,
                         (hipStream_t)stream), "drift");
  return NBODY_OK;
}

int nbody_step(nbody_ctx *c, int64_t n, double *xm, double *v, const double *thr, int32_t nsteps,
               int32_t *pairs, int64_t cap, int64_t *count, int64_t *step_counts, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  TRY(check_dev(c, thr, "thr", false));
  if (nsteps < 0) return fail(c, NBODY_E_INVAL, "nsteps < 0");
  const bool emit = count != nullptr;
  if (emit) {
    TRY(check_dev(c, count, "count", true));
    if (cap < 0) return fail(c, NBODY_E_INVAL, "cap < 0");
    if (cap > 0) TRY(check_dev(c, pairs, "pairs", true));
  }
  TRY(check_dev(c, step_counts, "step_counts", false));
  const bool counting = step_counts != nullptr;
  unsigned long long *sc = (unsigned long long *)step_counts;
  hipStream_t st = (hipStream_t)stream;
  if (counting)
    HIPCHK(c, hipMemsetAsync(step_counts, 0, ((size_t)nsteps + 1) * sizeof(int64_t), st), "memset");
  const nbody_params &p = c->p;
  const int N = (int)n;
  if (!thr) {
    double *t = (double *)ensure(c, B_THR, (size_t)n * sizeof(double4));
    if (!t) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (thresholds)");
    TRY(nbody_rcrit(c, n, xm, v, t, stream));
    thr = t;
  }
  const int nbf = fin_blocks(n);   // momentum partials (one per 64 bodies)
  double4 *momA = (double4 *)ensure(c, B_MOM_A, (size_t)nbf * sizeof(double4));
  double4 *momB = (double4 *)ensure(c, B_MOM_B, (size_t)nbf * sizeof(double4));
  if (!momA || !momB) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (momentum)");
  KickArgs a;
  TRY(make_kick_args(c, N, xm, thr, true, false, emit || counting, a));
  // counting-only evaluations: the emission path with no partner slots (partners counted, not kept)
  KickArgs ac = a;
  ac.R = 0;
  ac.rowbuf = nullptr;
  ac.rowsum = nullptr;   // no emission follows these launches
  ac.rowmask = nullptr;
  const bool split = p.precision == NBODY_PREC_SPLIT;
  const double h = 0.5 * p.dt;
  const double mu = p.G * p.m0;
  double4 *X = (double4 *)xm;
  double4 *Vv = (double4 *)v;
  TRY(locality(c, N, X, st, &a.perm));
  TRY(mass_check(c, N, X, st, &a.uni));
  ac.perm = a.perm;
  ac.uni = a.uni;
  if (nsteps == 0) {
    if (emit || counting) HIPCHK(c, launch_pairs(emit ? a : ac, false, true, false, false, st), "step pairs");
    if (counting)
      HIPCHK(c, launch_finalize(nullptr, nullptr, a.nchunk, N, p.G, h, 1, X, nullptr, nullptr, nullptr,
                                nullptr, st, a.cnt, sc), "step count");
    if (emit) return emit_list(c, a, pairs, cap, count, st);
    return NBODY_OK;
  }
  HIPCHK(c, launch_pairs(counting ? ac : a, true, counting, false, split, st), "step pairs");
  HIPCHK(c, launch_finalize(a.part, nullptr, a.nchunk, N, p.G, h, 1, X, Vv, nullptr, nullptr, momA, st,
                            counting ? a.cnt : nullptr, sc), "step finalize");
  for (int s = 1; s <= nsteps; ++s) {
    HIPCHK(c, launch_jump_drift(X, Vv, momA, nbf, N, h, p.dt, p.m0, mu, nullptr, momB, st), "jump+drift");
    HIPCHK(c, launch_jump(X, momB, nbf, N, h, p.m0, st), "jump");
    if (a.perm && s % c->locality_every == 0) {
      TRY(locality(c, N, X, st, &a.perm));
      ac.perm = a.perm;
    }
    const bool last = s == nsteps;
    const bool em = last && emit;
    HIPCHK(c, launch_pairs(em ? a : ac, true, em || counting, false, split, st), "step pairs");
    HIPCHK(c, launch_finalize(a.part, nullptr, a.nchunk, N, p.G, h, last ? 1 : 2, X, Vv, nullptr,
                              nullptr, momA, st, counting ? a.cnt : nullptr, counting ? sc + s : nullptr),
           "step finalize");
  }
  if (emit) return emit_list(c, a, pairs, cap, count, st);
  return NBODY_OK;
}

int nbody_encounter_groups(nbody_ctx *c, int64_t n, const int32_t *pairs, int64_t cap, const int64_t *count,
                           int32_t *labels, int64_t *out, void *stream) {
  TRY(check_n(c, n));
  if (cap < 0) return fail(c, NBODY_E_INVAL, "cap < 0");
  if (cap > 0) TRY(check_dev(c, pairs, "pairs", true));
  TRY(check_dev(c, count, "count", true));
  TRY(check_dev(c, labels, "labels", true));
  TRY(check_dev(c, out, "out", true));
  int *gsize = (int *)ensure(c, B_GSIZE, (size_t)n * sizeof(int));
  if (!gsize) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (groups)");
  const int64_t want = (cap + kBlock - 1) / kBlock;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, 4096));
  if (n <= kGroupsSmall)
    HIPCHK(c, launch_groups_small(pairs, cap, count, (int)n, labels, gsize, out, (hipStream_t)stream,
                                  nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr), "groups");
  else
    HIPCHK(c, launch_groups(pairs, cap, count, (int)n, labels, gsize, nullptr, nullptr, out, blocks,
                            (hipStream_t)stream), "groups");
  return NBODY_OK;
}

int nbody_drift_groups(nbody_ctx *c, int64_t n, double *xm, double *v, const double *thr, const int32_t *labels,
                       double h, const nbody_collisions *col, int64_t *stats, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  TRY(check_dev(c, thr, "thr", true));
  TRY(check_dev(c, labels, "labels", true));
  TRY(check_dev(c, stats, "stats", true));
  CeCollide cc;
  TRY(collide_args(c, (int)n, col, cc));
  hipStream_t st = (hipStream_t)stream;
  GroupBufs g;
  TRY(group_bufs(c, (int)n, g));
  HIPCHK(c, hipMemsetAsync(stats, 0, 6 * sizeof(int64_t), st), "memset");
  if (cc.count) HIPCHK(c, hipMemsetAsync(cc.count, 0, sizeof(int64_t), st), "memset");
  TRY(ce_drift(c, (int)n, (double4 *)xm, (double4 *)v, (const double4 *)thr, labels, g, h,
               (unsigned long long *)stats, cc, st));
  // bodies in no group: Kepler orbits (g.in marks the group members)
  HIPCHK(c, launch_drift((double4 *)xm, (double4 *)v, (int)n, h, c->p.G * c->p.m0, nullptr, st, g.in), "drift");
  return NBODY_OK;
}

int nbody_step_hybrid(nbody_ctx *c, int64_t n, double *xm, double *v, const double *thr, int32_t nsteps,
                      const nbody_levels *lv, const nbody_collisions *col, int64_t *stats, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  TRY(check_dev(c, thr, "thr", false));
  TRY(check_dev(c, stats, "stats", true));
  if (nsteps < 0) return fail(c, NBODY_E_INVAL, "nsteps < 0");
  if (c->p.precision != NBODY_PREC_F64) return fail(c, NBODY_E_INVAL, "the hybrid step runs in binary64");
  const int L = lv ? lv->levels : 0;
  const int sub = lv ? lv->substeps : 1;
  const double margin = lv ? lv->margin : 0.0;
  if (L < 0 || L >= kMaxLevels) return fail(c, NBODY_E_INVAL, "levels must be 0..%d", kMaxLevels - 1);
  if (L > 0 && sub < 1) return fail(c, NBODY_E_INVAL, "substeps must be >= 1");
  if (!(margin >= 0.0) || !std::isfinite(margin)) return fail(c, NBODY_E_INVAL, "margin must be finite and >= 0");
  CeCollide cc;
  TRY(collide_args(c, (int)n, col, cc));
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(c, hipMemsetAsync(stats, 0, 6 * sizeof(int64_t), st), "memset");
  if (cc.count) HIPCHK(c, hipMemsetAsync(cc.count, 0, sizeof(int64_t), st), "memset");
  if (nsteps == 0) return NBODY_OK;
  const nbody_params &p = c->p;
  const int N = (int)n;
  if (!thr) {
    double *t = (double *)ensure(c, B_THR, (size_t)n * sizeof(double4));
    if (!t) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (thresholds)");
    TRY(nbody_rcrit(c, n, xm, v, t, stream));
    thr = t;
  }
  const int nbf = fin_blocks(n);
  double4 *momA = (double4 *)ensure(c, B_MOM_A, (size_t)nbf * sizeof(double4));
  double4 *momB = (double4 *)ensure(c, B_MOM_B, (size_t)nbf * sizeof(double4));
  // the encounter list of every force evaluation, its groups and their member lists
  const int64_t cap = std::max<int64_t>(16 * n, 65536);
  int32_t *lpairs = (int32_t *)ensure(c, B_HPAIRS, (size_t)cap * 2 * sizeof(int32_t));
  int64_t *lcount = (int64_t *)ensure(c, B_HCOUNT, sizeof(int64_t));
  int32_t *labels = (int32_t *)ensure(c, B_HLAB, (size_t)n * sizeof(int32_t));
  if (!momA || !momB || !lpairs || !lcount || !labels)
    return fail(c, NBODY_E_NOMEM, "workspace allocation failed (hybrid step)");
  GroupBufs g;
  TRY(group_bufs(c, N, g));
  // with levels and a margin, the pair loop lists the pairs within (1 + margin) rc
  const double *thr_list = thr;
  if (L > 0 && margin > 0.0) {
    double4 *te = (double4 *)ensure(c, B_ETHR, (size_t)n * sizeof(double4));
    if (!te) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (list thresholds)");
    const double f = 1.0 + margin, f2 = f * f, f6 = (f2 * f2) * f2;
    HIPCHK(c, launch_thr_scale((const double4 *)thr, N, f2, f6, te, st), "list thresholds");
    thr_list = (const double *)te;
  }
  KickArgs a;
  TRY(make_kick_args(c, N, xm, thr_list, true, false, true, a));
  double4 *X = (double4 *)xm;
  double4 *Vv = (double4 *)v;
  const double4 *T = (const double4 *)thr;
  unsigned long long *S = (unsigned long long *)stats;
  const double h = 0.5 * p.dt;
  const double mu = p.G * p.m0;
  TRY(locality(c, N, X, st, &a.perm));
  TRY(mass_check(c, N, X, st, &a.uni));
  const int ublocks = (int)std::min<int64_t>(4096, (cap + kBlock - 1) / kBlock);
  // intermediate changeover levels: thresholds at dt / sub^l (fixed for the call), the symmetric
  // adjacency of each step's close pairs, and a drift mask
  LevelThr lt{};
  lt.thr[0] = T;
  lt.nl = L + 1;
  LevelAdj la{};
  int *lskip = nullptr;
  // above kGroupsSmall bodies the deepest level's groups come from the unions of the level kick
  // before each of its drifts (forest in labels), one flattening launch with member slices of
  // fixed length, and the drift launch that resets the forest; the group sizes and counters
  // alternate between two buffers (lgs, lcnt) so that the drift can clear the next pair while it
  // reads the current one
  const bool small = N <= kGroupsSmall;
  int *lgs[2] = {g.gsize, nullptr}, *lcnt[2] = {g.counter, nullptr}, *lslice = nullptr;
  int lpar = 0;
  if (L > 0) {
    double4 *lthr = (double4 *)ensure(c, B_LTHR, (size_t)L * n * sizeof(double4));
    la.deg = (int *)ensure(c, B_ADEG, (size_t)n * sizeof(int));
    la.off = (int *)ensure(c, B_AOFF, (size_t)n * sizeof(int));
    la.fill = (int *)ensure(c, B_AFILL, (size_t)n * sizeof(int));
    la.adj = (int *)ensure(c, B_ADJ, (size_t)cap * 2 * sizeof(int));
    la.total = (int *)ensure(c, B_ATOT, 2 * sizeof(int));
    la.longv = (int *)ensure(c, B_ALONG, (size_t)n * sizeof(int));
    lskip = (int *)ensure(c, B_LSKIP, (size_t)n * sizeof(int));
    if (!lthr || !la.deg || !la.off || !la.fill || !la.adj || !la.total || !la.longv || !lskip)
      return fail(c, NBODY_E_NOMEM, "workspace allocation failed (changeover levels)");
    if (!small) {
      lgs[1] = (int *)ensure(c, B_GSIZE2, (size_t)n * sizeof(int));
      lcnt[1] = (int *)ensure(c, B_GCNT2, kGroupCounters * sizeof(int));
      lslice = (int *)ensure(c, B_GSLICE, (size_t)n * kLevelSlice * sizeof(int));
      if (!lgs[1] || !lcnt[1] || !lslice)
        return fail(c, NBODY_E_NOMEM, "workspace allocation failed (changeover levels)");
      for (int q = 0; q < 2; ++q)
        HIPCHK(c, launch_groups_init(labels, lgs[q], N, lcnt[q], st), "level forest");
    }
    const double cH = ((p.n1 * p.n1 * p.n1) * (p.n1 * p.n1 * p.n1)) / 9.0;
    double dtl = p.dt;
    for (int l = 1; l <= L; ++l) {
      dtl = dtl / sub;
      const double t = p.n2 * dtl;
      HIPCHK(c, launch_rcrit(X, Vv, lthr + (size_t)(l - 1) * n, N, p.m0, cH, t * t, p.n1, t, st), "level rcrit");
      lt.thr[l] = lthr + (size_t)(l - 1) * n;
    }
  }
  // groups of the list at the current kick positions (and, with levels, its adjacency); a list
  // longer than cap is counted in stats[5]. Up to kGroupsSmall bodies the groups and their member
  // lists come from one one-workgroup launch.
  auto groups_now = [&]() -> int {
    TRY(emit_list(c, a, lpairs, cap, lcount, st, S + 5));
    if (L == 0 && small)
      HIPCHK(c, launch_groups_small(lpairs, cap, lcount, N, labels, g.gsize, nullptr, st, nullptr, nullptr,
                                    g.in, g.gstart, g.gmem, g.groot, g.counter), "groups");
    else if (L == 0)
      HIPCHK(c, launch_groups(lpairs, cap, lcount, N, labels, g.gsize, g.gfill, g.counter, nullptr, ublocks,
                              st), "groups");
    else
      HIPCHK(c, launch_adjacency(lpairs, cap, lcount, N, la, st), "adjacency");
    return NBODY_OK;
  };
  int step = 0;
  // level-l drift over tau of the bodies with close partners: at the deepest level the groups of
  // the level-L close pairs go through the close-encounter integrator and the others follow Kepler
  // orbits; above it, sub substeps of kick / drift_{l+1} / kick
  std::function<int(int, double)> drift_levels = [&](int l, double tau) -> int {
    if (l == L) {
      // the groups, their member lists and the mask of the bodies that drift on Kepler orbits
      cc.step = step;
      if (small) {
        HIPCHK(c, launch_groups_small(lpairs, cap, lcount, N, labels, g.gsize, nullptr, st, X, lt.thr[L], g.in,
                                      g.gstart, g.gmem, g.groot, g.counter, la.deg, lskip), "level groups");
        HIPCHK(c, launch_ce_drift(X, Vv, T, g.gmem, g.gstart, g.gsize, g.groot, g.counter, N / 2 + 1, p.G,
                                  p.m0, p.f_in, tau, kCeTol, S, cc, lt, st), "close-encounter drift");
        HIPCHK(c, launch_drift(X, Vv, N, tau, mu, nullptr, st, lskip), "level drift");
      } else {
        // the forest in labels holds the unions of the level kick just before
        HIPCHK(c, launch_level_groups(la.deg, N, labels, lgs[lpar], g.gstart, lslice, g.groot, lcnt[lpar], st),
               "level groups");
        HIPCHK(c, launch_ce_drift(X, Vv, T, lslice, g.gstart, lgs[lpar], g.groot, lcnt[lpar], N / 2 + 1, p.G,
                                  p.m0, p.f_in, tau, kCeTol, S, cc, lt, st, kLevelSlice),
               "close-encounter drift");
        HIPCHK(c, launch_level_drift(X, Vv, N, tau, mu, la.deg, labels, lgs[lpar], lgs[lpar ^ 1], lcnt[lpar ^ 1],
                                     st), "level drift");
        lpar ^= 1;
      }
      return NBODY_OK;
    }
    // the closing half kick of a substep and the opening half kick of the next act at the same
    // positions: one kick over the whole substep length. A kick followed by a deepest-level drift
    // also joins that drift's groups (above kGroupsSmall bodies).
    const double ts = tau / sub;
    int *uf = (l + 1 == L && !small) ? labels : nullptr;
    HIPCHK(c, launch_level_kick(X, Vv, la, N, lt, l + 1, p.G, p.f_in, 0.5 * ts, st, uf), "level kick");
    for (int k = 0; k < sub; ++k) {
      TRY(drift_levels(l + 1, ts));
      HIPCHK(c, launch_level_kick(X, Vv, la, N, lt, l + 1, p.G, p.f_in, k + 1 < sub ? ts : 0.5 * ts, st,
                                  k + 1 < sub ? uf : nullptr), "level kick");
    }
    return NBODY_OK;
  };
  HIPCHK(c, launch_pairs(a, true, true, false, false, st), "hybrid pairs");
  HIPCHK(c, launch_finalize(a.part, nullptr, a.nchunk, N, p.G, h, 1, X, Vv, nullptr, nullptr, momA, st),
         "hybrid finalize");
  TRY(groups_now());
  for (int s = 1; s <= nsteps; ++s) {
    step = s - 1;
    if (L == 0) {
      if (!small)
        HIPCHK(c, launch_group_lists(labels, N, g.in, g.gsize, g.gstart, g.gfill, g.gmem, g.groot, g.counter,
                                     true, st), "group lists");
      // first jump for all; Kepler drift for the bodies in no group
      HIPCHK(c, launch_jump_drift(X, Vv, momA, nbf, N, h, p.dt, p.m0, mu, nullptr, momB, st, nullptr, nullptr,
                                  g.in), "jump+drift");
      cc.step = step;
      HIPCHK(c, launch_ce_drift(X, Vv, T, g.gmem, g.gstart, g.gsize, g.groot, g.counter, N / 2 + 1, p.G, p.m0,
                                p.f_in, p.dt, kCeTol, S, cc, lt, st), "close-encounter drift");
    } else {
      // first jump for all; Kepler drift for the bodies without close partners; the others
      // through the levels
      HIPCHK(c, launch_level_mask(la.deg, nullptr, N, lskip, st), "level mask");
      HIPCHK(c, launch_jump_drift(X, Vv, momA, nbf, N, h, p.dt, p.m0, mu, nullptr, momB, st, nullptr, nullptr,
                                  lskip), "jump+drift");
      TRY(drift_levels(0, p.dt));
    }
    // mergers change masses: the equal-mass flag of the pair kernel is taken again
    if (cc.radius) TRY(mass_check(c, N, X, st, &a.uni));
    if (N <= kJumpSmall) {
      HIPCHK(c, launch_momentum_jump_small(X, Vv, N, h, p.m0, st), "momentum + jump");
    } else {
      HIPCHK(c, launch_momentum(X, Vv, N, momB, st), "momentum");
      HIPCHK(c, launch_jump(X, momB, nbf, N, h, p.m0, st), "jump");
    }
    if (a.perm && s % c->locality_every == 0) TRY(locality(c, N, X, st, &a.perm));
    const bool last = s == nsteps;
    HIPCHK(c, launch_pairs(a, true, !last, false, false, st), "hybrid pairs");
    HIPCHK(c, launch_finalize(a.part, nullptr, a.nchunk, N, p.G, h, last ? 1 : 2, X, Vv, nullptr, nullptr,
                              momA, st), "hybrid finalize");
    if (!last) TRY(groups_now());
  }
  return NBODY_OK;
}

int nbody_validate(nbody_ctx *c, int64_t n, const double *xm, const double *v, int64_t *result,
                   void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  TRY(check_dev(c, result, "result", true));
  unsigned long long *key = (unsigned long long *)ensure(c, B_VKEY, sizeof(unsigned long long));
  if (!key) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (validate)");
  HIPCHK(c, launch_validate((const double4 *)xm, (const double4 *)v, (int)n, key, result, (hipStream_t)stream),
         "validate");
  return NBODY_OK;
}

int nbody_energy(nbody_ctx *c, int64_t n, const double *xm, const double *v, const double *thr,
                 double *out, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  TRY(check_dev(c, thr, "thr", true));
  TRY(check_dev(c, out, "out", true));
  const int nb = nblocks(n);
  double4 *ep = (double4 *)ensure(c, B_EPARTS, (size_t)nb * 10 * sizeof(double));
  if (!ep) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (energy)");
  HIPCHK(c, launch_energy((const double4 *)xm, (const double4 *)v, (const double4 *)thr, (int)n, c->p.G,
                          c->p.m0, c->p.f_in, ep, out, (hipStream_t)stream), "energy");
  return NBODY_OK;
}

int nbody_kick_vjp(nbody_ctx *c, int64_t n, const double *xm, const double *thr, double h,
                   const double *lam_v, double *lam_x, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, thr, "thr", true));
  TRY(check_dev(c, lam_v, "lam_v", true));
  TRY(check_dev(c, lam_x, "lam_x", true));
  const double2 *uni = nullptr;
  TRY(mass_check(c, (int)n, (const double4 *)xm, (hipStream_t)stream, &uni));
  return kick_vjp(c, (int)n, (const double4 *)xm, (const double4 *)thr, uni, (const double4 *)lam_v, h,
                  (double4 *)lam_x, (hipStream_t)stream);
}

int nbody_jump_vjp(nbody_ctx *c, int64_t n, const double *xm, const double *v, double h, double *lam_x,
                   double *lam_v, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  TRY(check_dev(c, lam_x, "lam_x", true));
  TRY(check_dev(c, lam_v, "lam_v", true));
  return jump_vjp(c, (int)n, (const double4 *)xm, (const double4 *)v, h, (double4 *)lam_x, (double4 *)lam_v,
                  (hipStream_t)stream);
}

int nbody_drift_vjp(nbody_ctx *c, int64_t n, const double *xm, const double *v, double h, double *lam_x,
                    double *lam_v, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  TRY(check_dev(c, lam_x, "lam_x", true));
  TRY(check_dev(c, lam_v, "lam_v", true));
  HIPCHK(c, launch_drift_vjp((const double4 *)xm, (const double4 *)v, (int)n, h, c->p.G * c->p.m0,
                             (double4 *)lam_x, (double4 *)lam_v, (hipStream_t)stream), "drift vjp");
  return NBODY_OK;
}

int nbody_step_vjp(nbody_ctx *c, int64_t n, const double *xm0, const double *v0, const double *thr,
                   int32_t nsteps, double *lam_x, double *lam_v, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm0, "xm0", true));
  TRY(check_dev(c, v0, "v0", true));
  TRY(check_dev(c, thr, "thr", true));
  TRY(check_dev(c, lam_x, "lam_x", true));
  TRY(check_dev(c, lam_v, "lam_v", true));
  if (nsteps < 0) return fail(c, NBODY_E_INVAL, "nsteps < 0");
  if (nsteps == 0) return NBODY_OK;
  hipStream_t st = (hipStream_t)stream;
  const nbody_params &p = c->p;
  const int N = (int)n;
  const size_t bytes = (size_t)n * sizeof(double4);
  // per step s: X_s (positions at its start), X1_s (before the drift), V1_s (after the first
  // half kick), V2_s (after the drift); plus the final positions
  double4 *S = (double4 *)ensure(c, B_ADJ_STATES, bytes * (4 * (size_t)nsteps + 1));
  double4 *XA = (double4 *)ensure(c, B_XA, bytes);
  double4 *VA = (double4 *)ensure(c, B_VA, bytes);
  const int nbf = fin_blocks(n);   // momentum partials (one per 64 bodies)
  double4 *momA = (double4 *)ensure(c, B_MOM_A, (size_t)nbf * sizeof(double4));
  double4 *momB = (double4 *)ensure(c, B_MOM_B, (size_t)nbf * sizeof(double4));
  if (!S || !XA || !VA || !momA || !momB)
    return fail(c, NBODY_E_NOMEM, "workspace allocation failed (adjoint states)");
  auto Xs = [&](int s) { return S + (size_t)4 * s * N; };
  auto X1 = [&](int s) { return S + ((size_t)4 * s + 1) * N; };
  auto V1 = [&](int s) { return S + ((size_t)4 * s + 2) * N; };
  auto V2 = [&](int s) { return S + ((size_t)4 * s + 3) * N; };
  double4 *Xend = S + (size_t)4 * nsteps * N;
  const double4 *T = (const double4 *)thr;
  const double h = 0.5 * p.dt;
  const bool split = p.precision == NBODY_PREC_SPLIT;
  // replay of the segment with the forward's own kernels in the forward's order (merged half
  // kicks, jump fused with the drift), so every recorded state equals the forward's bit for bit;
  // the kernels write the records as side outputs
  HIPCHK(c, hipMemcpyAsync(XA, xm0, bytes, hipMemcpyDeviceToDevice, st), "copy");
  HIPCHK(c, hipMemcpyAsync(VA, v0, bytes, hipMemcpyDeviceToDevice, st), "copy");
  HIPCHK(c, hipMemcpyAsync(Xs(0), xm0, bytes, hipMemcpyDeviceToDevice, st), "copy");
  KickArgs a;
  TRY(make_kick_args(c, N, (const double *)XA, thr, true, false, false, a));
  TRY(locality(c, N, XA, st, &a.perm));
  TRY(mass_check(c, N, XA, st, &a.uni));
  HIPCHK(c, launch_pairs(a, true, false, false, split, st), "pairs");
  HIPCHK(c, launch_finalize(a.part, nullptr, a.nchunk, N, p.G, h, 1, XA, VA, nullptr, nullptr, momA, st,
                            nullptr, nullptr, V1(0)), "finalize");
  for (int s = 0; s < nsteps; ++s) {
    HIPCHK(c, launch_jump_drift(XA, VA, momA, nbf, N, h, p.dt, p.m0, p.G * p.m0, nullptr, momB, st, X1(s),
                                V2(s)), "jump+drift");
    HIPCHK(c, launch_jump(XA, momB, nbf, N, h, p.m0, st, s + 1 < nsteps ? Xs(s + 1) : Xend), "jump");
    if (s + 1 < nsteps) {
      HIPCHK(c, launch_pairs(a, true, false, false, split, st), "pairs");
      HIPCHK(c, launch_finalize(a.part, nullptr, a.nchunk, N, p.G, h, 2, XA, VA, nullptr, nullptr, momA, st,
                                nullptr, nullptr, V1(s + 1)), "finalize");
    }
  }
  // reverse sweep: B2^T C2^T A^T C1^T B1^T per step. The first half kick of step s and the second
  // half kick of step s-1 sit at the same positions and see the same lam_v: one evaluation is
  // applied twice (identical bits to two evaluations).
  double4 *LX = (double4 *)lam_x, *LV = (double4 *)lam_v;
  // the segment's lane permutation (built at its start) serves every kick derivative: bodies
  // move little within a segment, and the permutation changes no result bit
  TRY(kick_vjp(c, N, Xend, T, a.uni, LV, h, LX, st, 1, a.perm));
  for (int s = nsteps - 1; s >= 0; --s) {
    TRY(jump_vjp(c, N, X1(s), V2(s), h, LX, LV, st));
    HIPCHK(c, launch_drift_vjp(X1(s), V1(s), N, p.dt, p.G * p.m0, LX, LV, st), "drift vjp");
    TRY(jump_vjp(c, N, X1(s), V1(s), h, LX, LV, st));
    TRY(kick_vjp(c, N, Xs(s), T, a.uni, LV, h, LX, st, s > 0 ? 2 : 1, a.perm));
  }
  return NBODY_OK;
}

int nbody_step_batched(nbody_ctx *c, int32_t nsys, const int64_t *offs, double *xm, double *v,
                       int32_t nsteps, uint64_t *npairs, void *stream) {
  if (!c) return NBODY_E_INVAL;
  TRY(check_offs(c, nsys, offs));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  TRY(check_dev(c, npairs, "npairs", false));
  if (nsteps < 0) return fail(c, NBODY_E_INVAL, "nsteps < 0");
  if (c->p.precision != NBODY_PREC_F64) return fail(c, NBODY_E_INVAL, "batched ensembles run in binary64");
  c->h_offs.assign(offs, offs + nsys + 1);
  return run_batched(c, nsys, c->tiles, (double4 *)xm, (double4 *)v, nsteps, (unsigned long long *)npairs,
                     (hipStream_t)stream);
}

// ------------------------------------------------------------------ small-N switch
// Paths: 0 = nbody_step's per-step launches; 1 and 2 = one persistent launch of the ensemble kernel
// for the single system (group tile, wave tile).
int run_step_path(nbody_ctx *c, int64_t n, double *xm, double *v, int32_t nsteps, int32_t path,
                  hipStream_t st) {
  if (path == 0)
    return nbody_step(c, n, xm, v, nullptr, nsteps, nullptr, 0, nullptr, nullptr, st);
  int32_t tiles[kBuckets];
  std::fill(tiles, tiles + kBuckets, path == 2 ? 1 : 0);
  c->h_offs.assign({0, n});
  return run_batched(c, 1, tiles, (double4 *)xm, (double4 *)v, nsteps, nullptr, st);
}

int nbody_autotune_step(nbody_ctx *c, int64_t n, const double *xm, const double *v, int32_t ntrial,
                        int32_t *choice, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  if (ntrial < 1) return fail(c, NBODY_E_INVAL, "ntrial < 1");
  hipStream_t st = (hipStream_t)stream;
  double *txm = (double *)ensure(c, B_T_XM, (size_t)n * sizeof(double4));
  double *tv = (double *)ensure(c, B_T_V, (size_t)n * sizeof(double4));
  if (!txm || !tv) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (autotune)");
  std::vector<int32_t> paths = {0};
  if (c->p.precision == NBODY_PREC_F64 && n <= (1 << (kBuckets + 5))) paths.push_back(1);
  if (c->p.precision == NBODY_PREC_F64 && n <= batched_max_wave_n()) paths.push_back(2);
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0), "event");
  HIPCHK(c, hipEventCreate(&e1), "event");
  std::vector<float> total(paths.size(), 0.f);
  int rc = NBODY_OK;
  // a warm-up run of every path, then the order a, b, c, c, b, a (cancels a linear clock drift)
  for (int pass = 0; pass < 3 && rc == NBODY_OK; ++pass)
    for (size_t k = 0; k < paths.size() && rc == NBODY_OK; ++k) {
      const size_t q = pass == 2 ? paths.size() - 1 - k : k;
      if ((rc = hipMemcpyAsync(txm, xm, (size_t)n * sizeof(double4), hipMemcpyDeviceToDevice, st)) != hipSuccess ||
          (rc = hipMemcpyAsync(tv, v, (size_t)n * sizeof(double4), hipMemcpyDeviceToDevice, st)) != hipSuccess) {
        rc = fail(c, NBODY_E_HIP, "copy");
        break;
      }
      if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(c, NBODY_E_HIP, "event"); break; }
      rc = run_step_path(c, n, txm, tv, ntrial, paths[q], st);
      if (rc != NBODY_OK) break;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = fail(c, NBODY_E_HIP, "event");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (pass > 0) total[q] += ms;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != NBODY_OK) return rc;
  size_t best = 0;
  for (size_t q = 1; q < paths.size(); ++q)
    if (total[q] < total[best]) best = q;
  c->step_path[n] = paths[best];
  if (choice) *choice = paths[best];
  return NBODY_OK;
}

int nbody_step_auto(nbody_ctx *c, int64_t n, double *xm, double *v, int32_t nsteps, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  if (nsteps < 0) return fail(c, NBODY_E_INVAL, "nsteps < 0");
  const auto it = c->step_path.find(n);
  // the persistent path integrates in binary64 only
  const int32_t path = it == c->step_path.end() || c->p.precision != NBODY_PREC_F64 ? 0 : it->second;
  return run_step_path(c, n, xm, v, nsteps, path, (hipStream_t)stream);
}

int nbody_autotune_batched(nbody_ctx *c, int32_t nsys, const int64_t *offs, const double *xm,
                           const double *v, int32_t nsteps, void *stream) {
  if (!c) return NBODY_E_INVAL;
  TRY(check_offs(c, nsys, offs));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, v, "v", true));
  if (nsteps < 1) return fail(c, NBODY_E_INVAL, "nsteps < 1");
  hipStream_t st = (hipStream_t)stream;
  c->h_offs.assign(offs, offs + nsys + 1);
  const int64_t tot = offs[nsys];
  double4 *txm = (double4 *)ensure(c, B_T_XM, (size_t)tot * sizeof(double4));
  double4 *tv = (double4 *)ensure(c, B_T_V, (size_t)tot * sizeof(double4));
  if (!txm || !tv) return fail(c, NBODY_E_NOMEM, "workspace allocation failed (autotune)");
  // classes present, and the largest system of each
  int64_t nmax[kBuckets] = {0};
  for (int32_t s = 0; s < nsys; ++s) {
    const int64_t n = offs[s + 1] - offs[s];
    const int b = size_class_host(n);
    nmax[b] = std::max(nmax[b], n);
  }
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0), "event");
  HIPCHK(c, hipEventCreate(&e1), "event");
  int rc = NBODY_OK;
  int32_t trial[kBuckets];
  std::copy(c->tiles, c->tiles + kBuckets, trial);
  // every class present is timed on its own systems (the others skipped; on scratch copies) with
  // each admissible tile code: one workgroup or one wave per system, one or two bodies per lane
  int only = -1;
  auto time_run = [&](double *ms_out) -> int {
    hipError_t e = hipMemcpyAsync(txm, xm, (size_t)tot * sizeof(double4), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(tv, v, (size_t)tot * sizeof(double4), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e != hipSuccess) return hip_fail(c, e, "autotune copy");
    TRY(run_batched(c, nsys, trial, txm, tv, nsteps, nullptr, st, only));
    float ms = 0.f;
    e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) return hip_fail(c, e, "autotune timing");
    *ms_out = ms;
    return NBODY_OK;
  };
  for (int b = kBuckets - 1; b >= 0 && rc == NBODY_OK; --b) {
    if (nmax[b] == 0) continue;
    const int incumbent = trial[b];
    int cand[kTileCodes], nc = 0;
    cand[nc++] = incumbent;
    for (int code = 0; code < kTileCodes; ++code)
      if (code != incumbent && (!(code & kTileWave) || nmax[b] <= batched_max_wave_n())) cand[nc++] = code;
    if (nc == 1) continue;
    only = b;
    // a warm-up run, then the candidates in order and in reverse order: the clock drifts during
    // the first runs, and the symmetric order cancels a linear drift
    double t_code[kTileCodes] = {0.0, 0.0, 0.0, 0.0}, ms = 0.0;
    trial[b] = incumbent;
    rc = time_run(&ms);
    for (int r = 0; r < 2 * nc && rc == NBODY_OK; ++r) {
      const int code = cand[r < nc ? r : 2 * nc - 1 - r];
      trial[b] = code;
      rc = time_run(&ms);
      t_code[code] += ms;
    }
    if (rc != NBODY_OK) break;
    // another code must win by more than the run-to-run spread (2 %) to replace the incumbent
    int best = incumbent;
    for (int q = 1; q < nc; ++q)
      if (t_code[cand[q]] < 0.98 * t_code[best]) best = cand[q];
    trial[b] = best;
  }
  // then the whole ensemble: the per-class choice against each code applied to every class (where
  // a class cannot take the wave tile, the same code without it), in symmetric order; another
  // set must win by more than 2 %. Classes interact through the queue's load balance, which the
  // per-class runs do not see.
  if (rc == NBODY_OK) {
    only = -1;
    int32_t sets[1 + kTileCodes][kBuckets];
    int ns = 0;
    std::copy(trial, trial + kBuckets, sets[ns++]);
    for (int code = 0; code < kTileCodes; ++code) {
      for (int b = 0; b < kBuckets; ++b)
        sets[ns][b] = (code & kTileWave) && nmax[b] > batched_max_wave_n() ? (code & ~kTileWave) : code;
      bool dup = false;
      for (int q = 0; q < ns && !dup; ++q) dup = std::equal(sets[q], sets[q] + kBuckets, sets[ns]);
      if (!dup) ++ns;
    }
    double t_set[1 + kTileCodes] = {0.0}, ms = 0.0;
    std::copy(sets[0], sets[0] + kBuckets, trial);
    rc = time_run(&ms);
    for (int r = 0; r < 2 * ns && rc == NBODY_OK; ++r) {
      const int q = r < ns ? r : 2 * ns - 1 - r;
      std::copy(sets[q], sets[q] + kBuckets, trial);
      rc = time_run(&ms);
      t_set[q] += ms;
    }
    int best = 0;
    for (int q = 1; q < ns; ++q)
      if (t_set[q] < 0.98 * t_set[best]) best = q;
    std::copy(sets[best], sets[best] + kBuckets, trial);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == NBODY_OK) {
    std::copy(trial, trial + kBuckets, c->tiles);
    c->tuned = true;
  }
  return rc;
}

int nbody_tune(nbody_ctx *c, const char *name, int64_t value) {
  if (!c || !name) return NBODY_E_INVAL;
  const std::string k(name);
  if (k == "locality_min_n" && value >= 1) c->locality_min_n = (int)std::min<int64_t>(value, INT32_MAX);
  else if (k == "locality_every" && value >= 1) c->locality_every = (int)std::min<int64_t>(value, INT32_MAX);
  else if (k == "emit_slots" && value >= 1 && value <= 4096) c->R = (int)value;
  else if (k == "target_waves" && value >= 64 && value <= (1 << 20)) c->target_waves = (int)value;
  else return fail(c, NBODY_E_INVAL, "unknown tuning key or value out of range: %s = %lld", name, (long long)value);
  return NBODY_OK;
}

int nbody_get_batched_tiles(const nbody_ctx *c, int32_t *tiles, int32_t n) {
  if (!c || !tiles || n < kBuckets) return NBODY_E_INVAL;
  for (int b = 0; b < kBuckets; ++b) tiles[b] = c->tiles[b];
  return kBuckets;
}

int nbody_set_batched_tiles(nbody_ctx *c, const int32_t *tiles, int32_t n) {
  if (!c || !tiles || n != kBuckets) return NBODY_E_INVAL;
  for (int b = 0; b < kBuckets; ++b)
    if (tiles[b] < 0 || tiles[b] >= kTileCodes)
      return fail(c, NBODY_E_INVAL, "tile code %d out of range (0 .. %d)", tiles[b], kTileCodes - 1);
  for (int b = 0; b < kBuckets; ++b) c->tiles[b] = tiles[b];
  return NBODY_OK;
}

int nbody_bench_pairs(nbody_ctx *c, int64_t n, const double *xm, const double *thr, int32_t reps,
                      double *avg_ms, void *stream) {
  TRY(check_n(c, n));
  TRY(check_dev(c, xm, "xm", true));
  TRY(check_dev(c, thr, "thr", true));
  if (reps <= 0 || !avg_ms) return fail(c, NBODY_E_INVAL, "reps <= 0 or avg_ms NULL");
  KickArgs a;
  TRY(make_kick_args(c, (int)n, xm, thr, true, false, false, a));
  hipStream_t st = (hipStream_t)stream;
  TRY(locality(c, (int)n, a.xm, st, &a.perm));
  TRY(mass_check(c, (int)n, a.xm, st, &a.uni));
  const bool split = c->p.precision == NBODY_PREC_SPLIT;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0), "event");
  HIPCHK(c, hipEventCreate(&e1), "event");
  hipError_t e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_pairs(a, true, false, false, split, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(c, e, "bench pairs");
  *avg_ms = (double)ms / reps;
  return NBODY_OK;
}

}  // extern "C"
