// Batched ensembles: many independent planetesimal systems of uneven size, each integrated for
// nsteps steps B C A C B, all in one persistent launch.
//
// Scheduling: workgroups take systems from an atomic queue ordered largest first (longest
// processing time first). A system runs with one of two tiles chosen per size class:
//   group tile - the eight waves of the workgroup share one system (up to 2048 bodies),
//   wave tile  - every wave owns a system of its own (up to 256 bodies).
// Once a workgroup meets a wave-tile system it stays in that mode: the queue is sorted, so
// everything after it is small as well.
//
// Group-tile balance: the kick of a system with rb row blocks of 64 bodies is cut into rb * C
// tiles (row block, j-chunk), C = 8 / gcd(rb, 8), so that every wave gets the same number of
// consecutive tiles. A wave accumulates the chunks of one row block in registers; a row block
// cut by a wave boundary leaves one partial sum per wave in a small per-workgroup scratch area
// and is completed after a barrier, partials added in wave (= j) order. The result depends on N
// only, never on which workgroup or wave runs the system.
//
// Positions live in LDS for the whole integration (the j-stream of the kick is an LDS broadcast:
// positions change inside the launch, so the scalar-load path of the single-system kernel, whose
// cache is not coherent with vector stores, is not used here). Velocities stay in HBM and are
// read and written only by the lane that owns the body.
#include "internal.hpp"
#include "kepler_core.hpp"

namespace nbk {
using namespace nbd;

constexpr int kBB = 512;                 // threads per workgroup of the batched kernel (8 wave64)
constexpr int kWaves = kBB / 64;
constexpr int kMaxGroupN = 2048;
constexpr int kMaxWaveN = 256;
static_assert(kWaves * kMaxWaveN == kMaxGroupN, "LDS regions of the two tiles coincide");
static_assert(kWaves == kBatchedWaves, "scratch sizing on the host");

struct BatchArgs {
  const int64_t *offs;   // [nsys + 1] body offsets
  const int32_t *order;  // [nsys] system ids, largest first
  const int32_t *cfg;    // [kBuckets] tile per size class: 1 = wave tile, 0 = group tile
  int nsys;
  int nsteps;
  double4 *xm;
  double4 *v;
  double4 *thr;          // workspace [sum N]
  double4 *part;         // workspace [grid][2 * kWaves][64]: partial sums of cut row blocks
  unsigned long long *npairs;  // [nsys] close pairs at the final positions (or null)
  unsigned *queue;
  double G, m0, dt, f_in, cH, cV, n1, n2dt, c15;
};

__device__ __forceinline__ int size_class(int n) {
  int b = 0;
  while (b < kBuckets - 1 && n > (64 << b)) ++b;
  return b;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <bool GROUP>
__device__ __forceinline__ void tile_sync() {
  if (GROUP) __syncthreads(); else wave_sync();
}

// Deterministic sum over the tile (all lanes of the tile receive the same bits): butterfly within
// each wave (commutative pairings give every lane the same value), then the wave results in
// wave order.
template <bool GROUP>
__device__ __forceinline__ void tile_sum3(double (&P)[3], double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int k = 0; k < 3; ++k) P[k] += __shfl_xor(P[k], o, 64);
  if (GROUP) {
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
      for (int k = 0; k < 3; ++k) red[3 * w + k] = P[k];
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
      double s = red[k];
      for (int q = 1; q < kWaves; ++q) s += red[3 * q + k];
      P[k] = s;
    }
    __syncthreads();
  }
}

// Smallest and largest mass over the tile's system (equal masses select the loop that applies m
// once after the sum).
template <bool GROUP>
__device__ __forceinline__ bool tile_equal_mass(const double4 *X, int N, double *red) {
  const int t = GROUP ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  const int nt = GROUP ? kBB : 64;
  double lo = X[0].w, hi = X[0].w;
  for (int i = t; i < N; i += nt) {
    lo = fmin(lo, X[i].w);
    hi = fmax(hi, X[i].w);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  if (GROUP) {
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[2 * w] = lo; red[2 * w + 1] = hi; }
    __syncthreads();
    for (int q = 0; q < kWaves; ++q) { lo = fmin(lo, red[2 * q]); hi = fmax(hi, red[2 * q + 1]); }
    __syncthreads();
  }
  return lo == hi;
}

// One pair (ii, j) of the LDS kick: adds the contribution of body j (position/mass pj, prefilter
// word tj) to acc.
template <bool UNI>
__device__ __forceinline__ void pair_lds(const double4 &xi, const double4 &pj, uint32_t tj, int j,
                                         const double4 *__restrict__ thr, int ii, bool valid,
                                         uint32_t tw, double f_in, double c15,
                                         double (&acc)[3], unsigned &npairs, bool count) {
  const uint32_t U = tw > tj ? tw : tj;
  const double dx = pj.x - xi.x, dy = pj.y - xi.y, dz = pj.z - xi.z;
  const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  double s = UNI ? rinv3(r2, c15) : m_rinv3(r2, pj.w, c15);
  if (hiword(r2) <= U) {
    if (j == ii) {
      s = 0.0;
    } else {
      const double4 ti = thr[ii];
      const double4 tq = thr[j];
      if (close_exact(r2, ti.y, tq.y, ti.z, tq.z)) {
        const double w = close_weight(r2, ti.x > tq.x ? ti.x : tq.x, f_in);
        s = UNI ? w : pj.w * w;
        if (count && valid && j > ii) ++npairs;
      }
    }
  }
  acc[0] = fma(s, dx, acc[0]);
  acc[1] = fma(s, dy, acc[1]);
  acc[2] = fma(s, dz, acc[2]);
}

// Adds to acc the accelerations (without G; without m when UNI) on body ii from bodies j0..j1-1
// in LDS, in ascending j. tw = wave maximum of the prefilter words of the wave's bodies. The
// j-bodies are read four at a time, so one LDS address serves all four.
template <bool UNI>
__device__ __forceinline__ void kick_rows(const double4 *X, const uint32_t *T,
                                          const double4 *__restrict__ thr, int ii, bool valid,
                                          uint32_t tw, int j0, int j1, double f_in, double c15,
                                          double (&acc)[3], unsigned &npairs,
                                          bool count) {
  const double4 xi = X[ii];
  // 1.5 held in a VGPR for the whole loop: one VOP3 instruction reads at most one scalar operand,
  // and the correction's fma already reads the j-body's data from SGPRs
  double c15v;
  asm volatile("v_mov_b64 %0, %1" : "=v"(c15v) : "s"(c15));
  int j = j0;
  for (; j + 4 <= j1; j += 4) {
    double4 p[4];
    uint32_t t[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      p[q] = X[j + q];
      t[q] = __builtin_amdgcn_readfirstlane(T[j + q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      pair_lds<UNI>(xi, p[q], t[q], j + q, thr, ii, valid, tw, f_in, c15v, acc, npairs, count);
  }
  for (; j < j1; ++j)
    pair_lds<UNI>(xi, X[j], __builtin_amdgcn_readfirstlane(T[j]), j, thr, ii, valid, tw, f_in, c15v,
                  acc, npairs, count);
}

// v += h G a (napply times) for body ii; adds m v to P.
template <bool UNI>
__device__ __forceinline__ void kick_apply(const BatchArgs &a, int64_t o, const double4 *X, int ii,
                                           double (&acc)[3], double h, int napply, double (&P)[3]) {
  if (UNI) {
    const double mu = X[0].w;
    acc[0] *= mu; acc[1] *= mu; acc[2] *= mu;
  }
  const double ax = a.G * acc[0], ay = a.G * acc[1], az = a.G * acc[2];
  double4 vi = a.v[o + ii];
  for (int k = 0; k < napply; ++k) {
    vi.x = vi.x + h * ax;
    vi.y = vi.y + h * ay;
    vi.z = vi.z + h * az;
  }
  a.v[o + ii] = vi;
  const double m = X[ii].w;
  P[0] += m * vi.x; P[1] += m * vi.y; P[2] += m * vi.z;
}

__device__ __forceinline__ uint32_t rows_tw(const uint32_t *T, int ii) {
  return __builtin_amdgcn_readfirstlane(wave_max_u32(T[ii]));
}

// Kick of a wave-tile system: the wave owns every row block.
template <bool UNI>
__device__ __forceinline__ void kick_wave(const BatchArgs &a, int64_t o, int N, const double4 *X,
                                          const uint32_t *T, double h, int napply, bool count,
                                          double (&P)[3], unsigned &npairs) {
  const int lane = threadIdx.x & 63;
  P[0] = P[1] = P[2] = 0.0;
  for (int r = 0; r * 64 < N; ++r) {
    const int i = r * 64 + lane;
    const bool valid = i < N;
    const int ii = valid ? i : N - 1;
    double acc[3] = {0.0, 0.0, 0.0};
    kick_rows<UNI>(X, T, a.thr + o, ii, valid, rows_tw(T, ii), 0, N, a.f_in, a.c15, acc,
                   npairs, count);
    if (valid) kick_apply<UNI>(a, o, X, ii, acc, h, napply, P);
  }
}

// Kick of a group-tile system: wave w takes tiles [w per, (w+1) per) of the rb * C tiles, tile
// t = (row block t / C, j-chunk t % C).
template <bool UNI>
__device__ __forceinline__ void kick_group(const BatchArgs &a, int64_t o, int N, const double4 *X,
                                           const uint32_t *T, double h, int napply, bool count,
                                           double (&P)[3], unsigned &npairs) {
  // wave index made provably uniform, so that the tile bounds and the j-loop live in SGPRs
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int rb = (N + 63) >> 6;
  const int low = rb & -rb;                                  // largest power of two dividing rb
  const int C = kWaves / (low < kWaves ? low : kWaves);      // kWaves / gcd(rb, kWaves)
  const int per = rb * C / kWaves;
  const int jc = (N + C - 1) / C;
  double4 *slot = a.part + (size_t)blockIdx.x * (2 * kWaves * 64);
  P[0] = P[1] = P[2] = 0.0;
  const int t0 = w * per, t1 = t0 + per;
  for (int r = t0 / C; r * C < t1; ++r) {
    const int c0 = max(t0, r * C) - r * C, c1 = min(t1, (r + 1) * C) - r * C;
    const int i = r * 64 + lane;
    const bool valid = i < N;
    const int ii = valid ? i : N - 1;
    double acc[3] = {0.0, 0.0, 0.0};
    kick_rows<UNI>(X, T, a.thr + o, ii, valid, rows_tw(T, ii), c0 * jc, min(N, c1 * jc), a.f_in,
                   a.c15, acc, npairs, count);
    if (c0 == 0 && c1 == C) {
      if (valid) kick_apply<UNI>(a, o, X, ii, acc, h, napply, P);
    } else {
      slot[(2 * w + (r == t0 / C ? 0 : 1)) * 64 + lane] = make_double4(acc[0], acc[1], acc[2], 0.0);
    }
  }
  __syncthreads();
  // row blocks cut by a wave boundary, in order; the k-th goes to wave k
  int k = 0, rprev = -1;
  for (int bnd = 1; bnd < kWaves; ++bnd) {
    const int tb = bnd * per;
    if (tb % C == 0) continue;
    const int r = tb / C;
    if (r == rprev) continue;
    rprev = r;
    if (k++ != w) continue;
    const int i = r * 64 + lane;
    const int wl = ((r + 1) * C - 1) / per;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int q = (r * C) / per; q <= wl; ++q) {
      const double4 s = slot[(2 * q + (r == (q * per) / C ? 0 : 1)) * 64 + lane];
      acc[0] += s.x; acc[1] += s.y; acc[2] += s.z;
    }
    if (i < N) kick_apply<UNI>(a, o, X, i, acc, h, napply, P);
  }
}

template <bool GROUP, bool UNI>
__device__ __forceinline__ void kick_system(const BatchArgs &a, int64_t o, int N, const double4 *X,
                                            const uint32_t *T, double h, int napply, bool count,
                                            double (&P)[3], unsigned &npairs) {
  if (GROUP) kick_group<UNI>(a, o, N, X, T, h, napply, count, P, npairs);
  else kick_wave<UNI>(a, o, N, X, T, h, napply, count, P, npairs);
}

template <bool GROUP, bool UNI>
__device__ void run_steps(const BatchArgs &a, int s, double4 *X, uint32_t *T, double *red);

template <bool GROUP>
__device__ void run_system(const BatchArgs &a, int s, double4 *X, uint32_t *T, double *red) {
  const int64_t o = a.offs[s];
  const int N = (int)(a.offs[s + 1] - o);
  const int t = GROUP ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  const int nt = GROUP ? kBB : 64;
  for (int i = t; i < N; i += nt) {
    const double4 p = a.xm[o + i];
    const double4 th = body_thresholds(p, a.v[o + i], a.m0, a.cH, a.cV, a.n1, a.n2dt);
    a.thr[o + i] = th;
    X[i] = p;
    T[i] = hiword(th.w);
  }
  tile_sync<GROUP>();
  if (tile_equal_mass<GROUP>(X, N, red)) run_steps<GROUP, true>(a, s, X, T, red);
  else run_steps<GROUP, false>(a, s, X, T, red);
}

template <bool GROUP, bool UNI>
__device__ void run_steps(const BatchArgs &a, int s, double4 *X, uint32_t *T, double *red) {
  const int64_t o = a.offs[s];
  const int N = (int)(a.offs[s + 1] - o);
  const int t = GROUP ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  const int nt = GROUP ? kBB : 64;
  const double h = 0.5 * a.dt;
  const double mu = a.G * a.m0;
  double P[3];
  unsigned npairs = 0;
  kick_system<GROUP, UNI>(a, o, N, X, T, h, 1, a.nsteps == 0 && a.npairs, P, npairs);
  for (int step = 1; step <= a.nsteps; ++step) {
    tile_sum3<GROUP>(P, red);
    const double s1x = h * (P[0] / a.m0), s1y = h * (P[1] / a.m0), s1z = h * (P[2] / a.m0);
    double Q[3] = {0.0, 0.0, 0.0};
    for (int i = t; i < N; i += nt) {
      double4 p = X[i];
      double4 q = a.v[o + i];
      p.x = p.x + s1x; p.y = p.y + s1y; p.z = p.z + s1z;
      kepler_advance(p.x, p.y, p.z, q.x, q.y, q.z, mu, a.dt);
      X[i] = p;
      a.v[o + i] = q;
      Q[0] += p.w * q.x; Q[1] += p.w * q.y; Q[2] += p.w * q.z;
    }
    tile_sum3<GROUP>(Q, red);
    const double s2x = h * (Q[0] / a.m0), s2y = h * (Q[1] / a.m0), s2z = h * (Q[2] / a.m0);
    for (int i = t; i < N; i += nt) {
      double4 p = X[i];
      p.x = p.x + s2x; p.y = p.y + s2y; p.z = p.z + s2z;
      X[i] = p;
    }
    tile_sync<GROUP>();
    const bool last = step == a.nsteps;
    kick_system<GROUP, UNI>(a, o, N, X, T, h, last ? 1 : 2, last && a.npairs, P, npairs);
  }
  for (int i = t; i < N; i += nt) a.xm[o + i] = X[i];
  if (a.npairs) {
    unsigned long long c = npairs;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(a.npairs + s, c);
  }
  tile_sync<GROUP>();
}

__device__ __forceinline__ int pop_wave(unsigned *queue) {
  unsigned idx = 0;
  if ((threadIdx.x & 63) == 0) idx = atomicAdd(queue, 1u);
  return (int)__builtin_amdgcn_readfirstlane(idx);
}

__global__ __launch_bounds__(kBB) __attribute__((amdgpu_waves_per_eu(4))) void k_batched(BatchArgs a) {
  __shared__ double4 X[kMaxGroupN];
  __shared__ uint32_t T[kMaxGroupN];
  __shared__ double red[3 * kWaves];
  __shared__ int sidx;
  const int w = threadIdx.x >> 6;
  int idx;
  // group phase
  for (;;) {
    if (threadIdx.x == 0) sidx = (int)atomicAdd(a.queue, 1u);
    __syncthreads();
    idx = sidx;
    __syncthreads();
    if (idx >= a.nsys) return;
    const int s = a.order[idx];
    const int N = (int)(a.offs[s + 1] - a.offs[s]);
    if (a.cfg[size_class(N)] == 1 && N <= kMaxWaveN) break;
    run_system<true>(a, s, X, T, red);
  }
  // wave phase: wave 0 runs the system just taken, the other waves take their own
  double4 *WX = X + w * kMaxWaveN;
  uint32_t *WT = T + w * kMaxWaveN;
  int my = w == 0 ? idx : pop_wave(a.queue);
  while (my < a.nsys) {
    run_system<false>(a, a.order[my], WX, WT, nullptr);
    my = pop_wave(a.queue);
  }
}

hipError_t launch_batched(const BatchLaunch &b, hipStream_t st) {
  BatchArgs a;
  a.offs = b.offs; a.order = b.order; a.cfg = b.cfg; a.nsys = b.nsys; a.nsteps = b.nsteps;
  a.xm = b.xm; a.v = b.v; a.thr = b.thr; a.part = b.part; a.npairs = b.npairs; a.queue = b.queue;
  a.G = b.G; a.m0 = b.m0; a.dt = b.dt; a.f_in = b.f_in; a.cH = b.cH; a.cV = b.cV; a.n1 = b.n1;
  a.n2dt = b.n2dt; a.c15 = 1.5;
  hipError_t e = hipMemsetAsync(b.queue, 0, sizeof(unsigned), st);
  if (e != hipSuccess) return e;
  if (b.npairs) {
    e = hipMemsetAsync(b.npairs, 0, (size_t)b.nsys * sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_batched, dim3(b.grid), dim3(kBB), 0, st, a);
  return hipGetLastError();
}

int batched_max_group_n() { return kMaxGroupN; }
int batched_max_wave_n() { return kMaxWaveN; }

hipError_t batched_occupancy(int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batched, kBB, 0);
}

}  // namespace nbk
