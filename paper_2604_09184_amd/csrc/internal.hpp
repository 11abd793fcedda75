// Internal interface between the C-ABI layer (capi.hip) and the kernel files.
// Device helpers shared by the kernels of this library.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "device.hpp"

namespace nbk {

// ------------------------------------------------------------------ device helpers
// x from the lane that DPP control CTRL names (within a 16-lane row), in two 32-bit moves.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// r^-1 to a few ulp: the hardware reciprocal square root (relative error about 2^-24) refined by
// the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + O(e^3), e = 1 - r2 y^2.
__device__ __forceinline__ double rinv_refined(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double e = fma(-r2, y * y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

// 1/d for a normal d: the hardware reciprocal refined by two Newton steps x <- x + x (1 - d x),
// each of which squares the relative error.
__device__ __forceinline__ double recip_refined(double d) {
  double x = __builtin_amdgcn_rcp(d);
  x = fma(x, fma(-d, x, 1.0), x);
  x = fma(x, fma(-d, x, 1.0), x);
  return x;
}

// Lock-free union-find on a forest in global memory where a parent index is never larger than its
// child (every root is the smallest index of its set). Reads, and the path-halving writes of find,
// are device-scope atomics: a hook made by another workgroup must be seen.
__device__ __forceinline__ int uf_parent(const int *p, int x) {
  return __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int uf_find(int *p, int x) {
  int px = uf_parent(p, x);
  while (px != x) {
    const int gx = uf_parent(p, px);
    if (gx != px)   // path halving: point x at its grandparent (still in its set, still smaller)
      __hip_atomic_store(p + x, gx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = px;
    px = gx;
  }
  return x;
}

// Joins the sets of i and j by hooking the larger root under the smaller with a compare-and-swap.
// Termination: parent[x] <= x always and a hook or a halving only lowers it, so every find walks a
// strictly decreasing chain; a failed compare-and-swap means another thread hooked the same root,
// which lowers it, so a pair retries at most as often as its roots are lowered.
__device__ __forceinline__ void uf_unite(int *p, int i, int j) {
  int ri = uf_find(p, i), rj = uf_find(p, j);
  while (ri != rj) {
    const int lo = ri < rj ? ri : rj, hi = ri < rj ? rj : ri;
    const int old = atomicCAS(p + hi, hi, lo);
    if (old == hi) break;
    // hi was hooked meanwhile: continue from the roots as they are now
    ri = uf_find(p, lo);
    rj = uf_find(p, old);
  }
}

struct KickArgs {
  const double4 *xm;
  const double4 *thr;
  const int *perm;   // lane -> body (null: identity)
  const double2 *uni;  // {1, m} if all masses equal m, else {0, 0} (null: not known)
  int n;
  int nchunk;     // number of j-chunks (S)
  int chunk;      // bodies per j-chunk
  double f_in;
  double4 *part;     // [S][n] partial accelerations
  double4 *part_ce;  // [S][n] partial close-encounter parts (or null)
  int *cnt;          // [S][n] close partners j > i per chunk (emission only)
  int *rowbuf;       // [S][R][n] partner indices (emission only)
  int R;
  // Emission launches followed by launch_emit, S <= 64 kRowMaskWords (may be null): per row the
  // total of cnt over the chunks and the mask of its chunks with partners, added by integer
  // atomics in the pair kernel (the same values in any order) and cleared by launch_emit.
  int *rowsum = nullptr;                 // [n]
  unsigned long long *rowmask = nullptr; // [n][kRowMaskWords]
};
constexpr int kRowMaskWords = 4;

// kick.hip
hipError_t launch_rcrit(const double4 *xm, const double4 *v, double4 *thr, int n, double m0,
                        double cH, double cV, double n1, double n2dt, hipStream_t st);
hipError_t launch_pairs(const KickArgs &a, bool force, bool emit, bool ce, bool split,
                        hipStream_t st);
hipError_t launch_finalize(const double4 *part, const double4 *part_ce, int S, int n, double G,
                           double h, int napply, const double4 *xm, double4 *v, double4 *acc,
                           double4 *acc_ce, double4 *mom, hipStream_t st, const int *cnt = nullptr,
                           unsigned long long *count_out = nullptr, double4 *v_rec = nullptr);
hipError_t launch_locality(const double4 *xm, int n, float2 *range_part, unsigned short *cell,
                           unsigned *count, unsigned *cursor, int *perm, hipStream_t st);
int locality_cells();
hipError_t launch_mass_check(const double4 *xm, int n, double2 *part, double2 *uni, hipStream_t st);
// The encounter list of the emission buffers, sorted by (i, j), and its length in *count (also
// beyond cap); *overflow (may be null) is incremented when the length exceeds cap. Lists of up to
// kEmitSmall bodies are built by one workgroup in one launch.
constexpr int kEmitSmall = 4096;
hipError_t launch_emit(const KickArgs &a, int32_t *pairs, int64_t cap, int64_t *count,
                       int64_t *rowtot, int64_t *bsum, hipStream_t st,
                       unsigned long long *overflow = nullptr);
hipError_t launch_validate(const double4 *xm, const double4 *v, int n, unsigned long long *key,
                           int64_t *out, hipStream_t st);
hipError_t launch_energy(const double4 *xm, const double4 *v, const double4 *thr, int n, double G,
                         double m0, double f_in, double4 *eparts, double *out, hipStream_t st);

// kepler.hip
hipError_t launch_momentum(const double4 *xm, const double4 *v, int n, double4 *mom, hipStream_t st);
hipError_t launch_jump(double4 *xm, const double4 *mom, int nb, int n, double h, double m0,
                       hipStream_t st, double4 *x_rec = nullptr);
// launch_momentum followed by launch_jump for up to kJumpSmall bodies, in one launch, with the
// same result bits.
constexpr int kJumpSmall = 4096;
hipError_t launch_momentum_jump_small(double4 *xm, const double4 *v, int n, double h, double m0,
                                      hipStream_t st);
hipError_t launch_jump_drift(double4 *xm, double4 *v, const double4 *mom_in, int nb, int n,
                             double hjump, double dt, double m0, double mu, uint32_t *status,
                             double4 *mom_out, hipStream_t st, double4 *x_rec = nullptr,
                             double4 *v_rec = nullptr, const int *skip = nullptr);
hipError_t launch_drift(double4 *xm, double4 *v, int n, double dt, double mu, uint32_t *status,
                        hipStream_t st, const int *skip = nullptr);

// ce.hip
// Member lists of the groups (gsize >= 2) of the labels: in[i], gstart/gmem slices, root list
// groot and counter[0] = groups. counted: gsize, gfill and counter come from launch_groups;
// otherwise they are computed from the labels here.
// With deg and skip given, also the drift mask of the deepest changeover level:
// skip[i] = !(deg[i] > 0 && !in[i]) (bodies with listed partners outside the groups drift on
// Kepler orbits there).
hipError_t launch_group_lists(const int *label, int n, int *in, int *gsize, int *gstart, int *gfill,
                              int *gmem, int *groot, int *counter, bool counted, hipStream_t st,
                              const int *deg = nullptr, int *skip = nullptr);
// Collisions inside the close-encounter drift: radius null = none. Mergers are appended to
// merges [cap][3] = {step, survivor, removed} and mtime [cap] (time within the drift); count is
// incremented once per merger, also beyond cap.
struct CeCollide {
  double *radius;
  double f;
  int32_t *merges;
  double *mtime;
  int64_t cap;
  unsigned long long *count;
  int step;
  int n;
};

// Critical radii of the changeover levels 0..nl-1 (level 0 is the step's thr); the pair term of
// the close-encounter drift is weighted by prod_l [1 - K_l].
constexpr int kMaxLevels = 5;
struct LevelThr {
  const double4 *thr[kMaxLevels];
  int nl;
};

// counter [kGroupCounters]: [0] groups, [1] member slots allocated, [2] queue of the drift kernel
// (zeroed by launch_groups, launch_group_lists or launch_level_drift).
// slice > 0: member lists of launch_level_groups (slices of fixed length); the members of a group
// above 64 bodies are then not drifted here (launch_level_drift drifts them).
constexpr int kGroupCounters = 8;
hipError_t launch_ce_drift(double4 *xm, double4 *v, const double4 *thr, const int *gmem,
                           const int *gstart, const int *gsize, const int *groot, int *counter,
                           int max_groups, double G, double m0, double f_in, double h, double tol,
                           unsigned long long *stats, const CeCollide &col, const LevelThr &lt,
                           hipStream_t st, int slice = 0);

// levels.hip: symmetric adjacency of a pair list (rows sorted by neighbour index), the level kicks
// over it and the masks of the level drifts.
// deg/off/fill [n]; adj [2 cap] (the neighbour per slot); total [2]: slots used and the number of
// rows in longv [n] (the rows the level kick gives a whole wave).
struct LevelAdj {
  int *deg, *off, *fill, *adj, *total, *longv;
};
hipError_t launch_adjacency(const int32_t *pairs, int64_t cap, const int64_t *count, int n,
                            const LevelAdj &g, hipStream_t st);
// With parent given, the kick also joins (uf_unite on parent, which must hold a forest) every
// listed pair that is close under level `level`'s exact predicate at the kick's positions: the
// groups of the deepest level's drift that follows.
hipError_t launch_level_kick(const double4 *xm, double4 *v, const LevelAdj &g, int n, const LevelThr &lt,
                             int level, double G, double f_in, double h, hipStream_t st,
                             int *parent = nullptr);
// Deepest-level groups from the forest of the kick's unions, for n above kGroupsSmall: every body
// with listed partners is flattened onto its root (parent becomes the labels) and counted in
// gsize; member slices of kLevelSlice slots at gstart[r] = r kLevelSlice (gmem [n kLevelSlice]);
// the roots of groups (two or more bodies) into groot, their number into counter[0].
constexpr int kLevelSlice = 64;
hipError_t launch_level_groups(const int *deg, int n, int *parent, int *gsize, int *gstart, int *gmem,
                               int *groot, int *counter, hipStream_t st);
// Kepler drift over dt of the bodies with listed partners outside the groups of 2..64 bodies
// (gsize of their label), then the forest reset for the next deepest-level drift: parent[i] = i,
// gsize_next and counter_next zeroed.
hipError_t launch_level_drift(double4 *xm, double4 *v, int n, double dt, double mu, const int *deg,
                              int *parent, const int *gsize, int *gsize_next, int *counter_next,
                              hipStream_t st);
// skip[i] = 1 unless body i has a listed partner (deg > 0) and is outside the groups (in == 0);
// with in null: skip[i] = (deg[i] > 0).
hipError_t launch_level_mask(const int *deg, const int *in, int n, int *skip, hipStream_t st);
hipError_t launch_thr_scale(const double4 *thr, int n, double f2, double f6, double4 *out, hipStream_t st);

// adjoint.hip
hipError_t launch_kick_vjp(const double4 *xm, const double4 *thr, const int *perm, const double2 *uni,
                           const double4 *lam_v, double h, double G, double f_in, int n, int S,
                           int chunk, int napply, double4 *part, double4 *lam_x, hipStream_t st);
hipError_t launch_jump_vjp(const double4 *xm, const double4 *v, double h, double m0, int n,
                           double4 *parts, double4 *lam_x, double4 *lam_v, hipStream_t st);
hipError_t launch_drift_vjp(const double4 *xm, const double4 *v, int n, double dt, double mu,
                            double4 *lam_x, double4 *lam_v, hipStream_t st);

// groups.hip
// Labels of the groups of a pair list (union-find), and gsize[root] = bodies with that root (a
// group when >= 2). gsize [n] is written; gfill [n] (may be null) zeroed and counter (may be null)
// zeroed for launch_group_lists; out (may be null): {groups, invalid pairs}.
hipError_t launch_groups(const int32_t *pairs, int64_t cap, const int64_t *count, int n,
                         int32_t *labels, int *gsize, int *gfill, int *counter, int64_t *out,
                         int union_blocks, hipStream_t st, const double4 *xm = nullptr,
                         const double4 *thr = nullptr);
// parent[i] = i, gsize zeroed and counter zeroed (a forest of singletons for launch_level_kick).
hipError_t launch_groups_init(int *parent, int *gsize, int n, int *counter, hipStream_t st);
// The same for n <= kGroupsSmall in one workgroup and one launch; with in non-null also the member
// lists of launch_group_lists (in, gstart, gmem, groot, counter). out (may be null) is written,
// not accumulated.
constexpr int kGroupsSmall = 4096;
hipError_t launch_groups_small(const int32_t *pairs, int64_t cap, const int64_t *count, int n,
                               int32_t *labels, int *gsize, int64_t *out, hipStream_t st,
                               const double4 *xm, const double4 *thr, int *in, int *gstart,
                               int *gmem, int *groot, int *counter, const int *deg = nullptr,
                               int *skip = nullptr);

// batched.hip
constexpr int kBuckets = 6;   // size classes: N <= 64, 128, 256, 512, 1024, 2048
constexpr int kBatchedWaves = 8;   // waves per workgroup of the batched kernel
// Tile code of a size class: bit 0 set = one wave per system (systems of at most 256 bodies),
// clear = one workgroup per system; bit 1 set = two bodies per lane in the kick, clear = one.
constexpr int kTileWave = 1, kTileIpl2 = 2, kTileCodes = 4;
struct BatchLaunch {
  const int64_t *offs;
  const int32_t *order;
  const int32_t *cfg;   // [kBuckets] tile codes
  int nsys, nsteps, grid;
  double4 *xm, *v, *thr;
  double4 *part;        // [grid][2 * kBatchedWaves][2][64]
  unsigned long long *npairs;
  unsigned *queue;
  double G, m0, dt, f_in, cH, cV, n1, n2dt;
};
hipError_t launch_batched(const BatchLaunch &b, hipStream_t st);
hipError_t batched_occupancy(int *blocks_per_cu);
int batched_max_group_n();
int batched_max_wave_n();

inline int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }
// momentum partials (and the workgroups of k_finalize and of the jump and drift kernels): one per
// 64 bodies
inline int fin_blocks(int64_t n) { return (int)((n + 63) / 64); }

}  // namespace nbk
