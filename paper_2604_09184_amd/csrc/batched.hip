// Batched ensembles: many independent planetesimal systems of uneven size, each integrated for
// nsteps steps B C A C B, all in one persistent launch.
//
// Scheduling: workgroups take systems from an atomic queue ordered largest first (longest
// processing time first). A system runs with the tile its size class's code names:
//   group tile - the eight waves of the workgroup share one system (up to 2048 bodies),
//   wave tile  - every wave owns a system of its own (up to 256 bodies),
// and, in either, one or two bodies per lane in the kick (two: each j-body read from LDS serves
// two pairs, half the LDS traffic per pair). Once a workgroup meets a wave-tile system it stays in
// that mode: the queue is sorted, so everything after it is small as well.
//
// Group-tile balance: the kick of a system with rb row blocks of 64 (or 128) bodies is cut into rb * C
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
constexpr int kMaxIpl = 2;               // bodies per lane of the kick: 1 or 2
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

// The close-pair part of one pair that passed the per-pair prefilter: the exact predicate and the
// changeover weight. Kept out of line: it is rarely taken, and inlined into the unrolled pair loop
// its temporaries would crowd out the registers of the common path.
struct CloseOut {
  double s;
  unsigned counted;
};

template <bool UNI>
__device__ __attribute__((noinline)) CloseOut close_lds(double r2, double s, double mj, int j, int ii,
                                                        bool valid, bool count,
                                                        const double4 *__restrict__ thr,
                                                        double f_in) {
  CloseOut o{s, 0u};
  if (j == ii) {
    o.s = 0.0;
    return o;
  }
  const double4 ti = thr[ii];
  const double4 tq = thr[j];
  if (close_exact(r2, ti.y, tq.y, ti.z, tq.z)) {
    const double w = close_weight(r2, ti.x > tq.x ? ti.x : tq.x, f_in);
    o.s = UNI ? w : mj * w;
    if (count && valid && j > ii) o.counted = 1u;
  }
  return o;
}

// One pair (ii, j) of the LDS kick: r^-3, and for a pair that passes the per-pair prefilter
// hi(r2) <= max(T_i, T_j) the close-pair part.
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
    const CloseOut o = close_lds<UNI>(r2, s, pj.w, j, ii, valid, count, thr, f_in);
    s = o.s;
    npairs += o.counted;
  }
  acc[0] = fma(s, dx, acc[0]);
  acc[1] = fma(s, dy, acc[1]);
  acc[2] = fma(s, dz, acc[2]);
}

// Adds to acc[k] the accelerations (without G; without m when UNI) on the bodies ii[k],
// k < IPL, of every lane from the bodies j0..j1-1 in LDS, in ascending j. Each j-body read from LDS
// (one broadcast address for the wave) serves IPL pairs per lane; the j-bodies are read 4 / IPL at
// a time. tw = wave maximum of the prefilter words of the lanes' bodies. (A block screen as in the
// single-system pair kernel does not pay here: a wave's bodies span a large part of a small
// system, so few j-blocks would pass it.)
template <bool UNI, int IPL>
__device__ __forceinline__ void kick_rows(const double4 *X, const uint32_t *T,
                                          const double4 *__restrict__ thr, const int (&ii)[IPL],
                                          const bool (&valid)[IPL], uint32_t tw, int j0, int j1,
                                          double f_in, double c15, double (&acc)[IPL][3],
                                          unsigned &npairs, bool count) {
  double4 xi[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) xi[k] = X[ii[k]];
  // 1.5 held in a VGPR for the whole loop: one VOP3 instruction reads at most one scalar operand
  double c15v;
  asm volatile("v_mov_b64 %0, %1" : "=v"(c15v) : "s"(c15));
  // JU j-bodies per iteration: four pairs per lane in flight
  constexpr int JU = 4 / IPL;
  int j = j0;
  for (; j + JU <= j1; j += JU) {
    double4 p[JU];
    uint32_t t[JU];
#pragma unroll
    for (int q = 0; q < JU; ++q) {
      p[q] = X[j + q];
      t[q] = __builtin_amdgcn_readfirstlane(T[j + q]);
    }
#pragma unroll
    for (int q = 0; q < JU; ++q)
#pragma unroll
      for (int k = 0; k < IPL; ++k)
        pair_lds<UNI>(xi[k], p[q], t[q], j + q, thr, ii[k], valid[k], tw, f_in, c15v, acc[k], npairs,
                      count);
  }
  for (; j < j1; ++j) {
    const double4 p = X[j];
    const uint32_t t = __builtin_amdgcn_readfirstlane(T[j]);
#pragma unroll
    for (int k = 0; k < IPL; ++k)
      pair_lds<UNI>(xi[k], p, t, j, thr, ii[k], valid[k], tw, f_in, c15v, acc[k], npairs, count);
  }
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

// The lane's bodies of row block r (IPL * 64 bodies): ii[k] = r IPL 64 + k 64 + lane (clamped to
// N - 1 past the end) and the wave maximum of their prefilter words.
template <int IPL>
__device__ __forceinline__ uint32_t row_bodies(const uint32_t *T, int N, int r, int (&ii)[IPL],
                                               bool (&valid)[IPL]) {
  const int lane = threadIdx.x & 63;
  uint32_t t = 0;
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
    const int i = (r * IPL + k) * 64 + lane;
    valid[k] = i < N;
    ii[k] = valid[k] ? i : N - 1;
    t = max(t, T[ii[k]]);
  }
  return __builtin_amdgcn_readfirstlane(wave_max_u32(t));
}

// Kick of a wave-tile system: the wave owns every row block.
template <bool UNI, int IPL>
__device__ __forceinline__ void kick_wave(const BatchArgs &a, int64_t o, int N, const double4 *X,
                                          const uint32_t *T, double h, int napply, bool count,
                                          double (&P)[3], unsigned &npairs) {
  P[0] = P[1] = P[2] = 0.0;
  for (int r = 0; r * IPL * 64 < N; ++r) {
    int ii[IPL];
    bool valid[IPL];
    const uint32_t tw = row_bodies<IPL>(T, N, r, ii, valid);
    double acc[IPL][3] = {};
    kick_rows<UNI, IPL>(X, T, a.thr + o, ii, valid, tw, 0, N, a.f_in, a.c15, acc, npairs, count);
#pragma unroll
    for (int k = 0; k < IPL; ++k)
      if (valid[k]) kick_apply<UNI>(a, o, X, ii[k], acc[k], h, napply, P);
  }
}

// Kick of a group-tile system: rb row blocks of IPL * 64 bodies; wave w takes tiles
// [w per, (w+1) per) of the rb * C tiles, tile t = (row block t / C, j-chunk t % C).
template <bool UNI, int IPL>
__device__ __forceinline__ void kick_group(const BatchArgs &a, int64_t o, int N, const double4 *X,
                                           const uint32_t *T, double h, int napply, bool count,
                                           double (&P)[3], unsigned &npairs) {
  // wave index made provably uniform, so that the tile bounds and the j-loop live in SGPRs
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int rb = (N + IPL * 64 - 1) / (IPL * 64);
  const int low = rb & -rb;                                  // largest power of two dividing rb
  const int C = kWaves / (low < kWaves ? low : kWaves);      // kWaves / gcd(rb, kWaves)
  const int per = rb * C / kWaves;
  const int jc = (N + C - 1) / C;
  double4 *slot = a.part + (size_t)blockIdx.x * (2 * kWaves * 64 * kMaxIpl);
  P[0] = P[1] = P[2] = 0.0;
  const int t0 = w * per, t1 = t0 + per;
  for (int r = t0 / C; r * C < t1; ++r) {
    const int c0 = max(t0, r * C) - r * C, c1 = min(t1, (r + 1) * C) - r * C;
    int ii[IPL];
    bool valid[IPL];
    const uint32_t tw = row_bodies<IPL>(T, N, r, ii, valid);
    double acc[IPL][3] = {};
    kick_rows<UNI, IPL>(X, T, a.thr + o, ii, valid, tw, c0 * jc, min(N, c1 * jc), a.f_in, a.c15,
                        acc, npairs, count);
    if (c0 == 0 && c1 == C) {
#pragma unroll
      for (int k = 0; k < IPL; ++k)
        if (valid[k]) kick_apply<UNI>(a, o, X, ii[k], acc[k], h, napply, P);
    } else {
#pragma unroll
      for (int k = 0; k < IPL; ++k)
        slot[((2 * w + (r == t0 / C ? 0 : 1)) * kMaxIpl + k) * 64 + lane] =
            make_double4(acc[k][0], acc[k][1], acc[k][2], 0.0);
    }
  }
  __syncthreads();
  // row blocks cut by a wave boundary, in order; the q-th goes to wave q
  int q = 0, rprev = -1;
  for (int bnd = 1; bnd < kWaves; ++bnd) {
    const int tb = bnd * per;
    if (tb % C == 0) continue;
    const int r = tb / C;
    if (r == rprev) continue;
    rprev = r;
    if (q++ != w) continue;
    const int wl = ((r + 1) * C - 1) / per;
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int i = (r * IPL + k) * 64 + lane;
      double acc[3] = {0.0, 0.0, 0.0};
      for (int u = (r * C) / per; u <= wl; ++u) {
        const double4 s = slot[((2 * u + (r == (u * per) / C ? 0 : 1)) * kMaxIpl + k) * 64 + lane];
        acc[0] += s.x; acc[1] += s.y; acc[2] += s.z;
      }
      if (i < N) kick_apply<UNI>(a, o, X, i, acc, h, napply, P);
    }
  }
}

template <bool GROUP, bool UNI, int IPL>
__device__ __forceinline__ void kick_system(const BatchArgs &a, int64_t o, int N, const double4 *X,
                                            const uint32_t *T, double h, int napply, bool count,
                                            double (&P)[3], unsigned &npairs) {
  if (GROUP) kick_group<UNI, IPL>(a, o, N, X, T, h, napply, count, P, npairs);
  else kick_wave<UNI, IPL>(a, o, N, X, T, h, napply, count, P, npairs);
}

template <bool GROUP, bool UNI, int IPL>
__device__ __forceinline__ void run_steps(const BatchArgs &a, int s, double4 *X, uint32_t *T, double *red);

template <bool GROUP, int IPL>
__device__ __forceinline__ void run_system(const BatchArgs &a, int s, double4 *X, uint32_t *T, double *red) {
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
  if (tile_equal_mass<GROUP>(X, N, red)) run_steps<GROUP, true, IPL>(a, s, X, T, red);
  else run_steps<GROUP, false, IPL>(a, s, X, T, red);
}

template <bool GROUP, bool UNI, int IPL>
__device__ __forceinline__ void run_steps(const BatchArgs &a, int s, double4 *X, uint32_t *T, double *red) {
  const int64_t o = a.offs[s];
  const int N = (int)(a.offs[s + 1] - o);
  const int t = GROUP ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  const int nt = GROUP ? kBB : 64;
  const double h = 0.5 * a.dt;
  const double mu = a.G * a.m0;
  double P[3];
  unsigned npairs = 0;
  kick_system<GROUP, UNI, IPL>(a, o, N, X, T, h, 1, a.nsteps == 0 && a.npairs, P, npairs);
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
    kick_system<GROUP, UNI, IPL>(a, o, N, X, T, h, last ? 1 : 2, last && a.npairs, P, npairs);
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
    const int cfg = a.cfg[size_class(N)];
    if ((cfg & kTileWave) && N <= kMaxWaveN) break;
    if (cfg & kTileIpl2) run_system<true, 2>(a, s, X, T, red);
    else run_system<true, 1>(a, s, X, T, red);
  }
  // wave phase: wave 0 runs the system just taken, the other waves take their own
  double4 *WX = X + w * kMaxWaveN;
  uint32_t *WT = T + w * kMaxWaveN;
  int my = w == 0 ? idx : pop_wave(a.queue);
  while (my < a.nsys) {
    const int s = a.order[my];
    const int N = (int)(a.offs[s + 1] - a.offs[s]);
    if (a.cfg[size_class(N)] & kTileIpl2) run_system<false, 2>(a, s, WX, WT, nullptr);
    else run_system<false, 1>(a, s, WX, WT, nullptr);
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
