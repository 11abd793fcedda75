// Batched ensembles: many independent planetesimal systems of uneven size, each integrated for
// nsteps steps B C A C B, all in one persistent launch.
//
// Scheduling: workgroups take systems from an atomic queue ordered largest first (longest
// processing time first). A system runs with one of two tiles chosen per size class:
//   group tile - the four waves of the workgroup share one system (up to 2048 bodies),
//   wave tile  - every wave owns a system of its own (up to 512 bodies).
// and I = 1 or 2 bodies per lane. Once a workgroup meets a wave-tile system it stays in that
// mode: the queue is sorted, so everything after it is small as well.
//
// Positions live in LDS for the whole integration (the j-stream of the kick is an LDS broadcast:
// positions change inside the launch, so the scalar-load path of the single-system kernel, whose
// cache is not coherent with vector stores, is not used here). Velocities stay in HBM and are
// read and written only by the lane that owns the body.
#include "internal.hpp"
#include "kepler_core.hpp"

namespace nbk {
using namespace nbd;

constexpr int kMaxGroupN = 2048;
constexpr int kMaxWaveN = 512;
constexpr int kWaves = kBlock / 64;
static_assert(kWaves * kMaxWaveN == kMaxGroupN, "LDS regions of the two tiles coincide");

struct BatchArgs {
  const int64_t *offs;   // [nsys + 1] body offsets
  const int32_t *order;  // [nsys] system ids, largest first
  const int32_t *cfg;    // [kBuckets] tile per size class: bit 0 wave tile, bit 1 two bodies per lane
  int nsys;
  int nsteps;
  int forced;            // >= 0: use this tile for every system (autotuning trials)
  double4 *xm;
  double4 *v;
  double4 *thr;          // workspace [sum N]
  unsigned long long *npairs;  // [nsys] close pairs at the final positions (or null)
  unsigned *queue;
  double G, m0, dt, f_in, cH, cV, n1, n2dt, c15, c1875;
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

// Deterministic sum over the tile (all lanes of the tile receive the same bits).
template <bool GROUP>
__device__ __forceinline__ void tile_sum3(double (&P)[3], double *red) {
  if (GROUP) {
    block_sum<3>(P, red);
  } else {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int k = 0; k < 3; ++k) P[k] += __shfl_xor(P[k], o, 64);
  }
}

// Accelerations (without G) of bodies ib + q*64 + lane, q < I, against all N bodies in LDS.
template <int I>
__device__ __forceinline__ void kick_block(const double4 *X, const uint32_t *T,
                                           const double4 *__restrict__ thr, int N, int ib,
                                           double f_in, double c15, double c1875, double (&acc)[I][3],
                                           int (&ii)[I], bool (&valid)[I], unsigned &npairs, bool count) {
  const int lane = threadIdx.x & 63;
  double4 xi[I];
  uint32_t tmax = 0;
#pragma unroll
  for (int q = 0; q < I; ++q) {
    const int i = ib + q * 64 + lane;
    valid[q] = i < N;
    ii[q] = valid[q] ? i : N - 1;
    xi[q] = X[ii[q]];
    const uint32_t t = T[ii[q]];
    tmax = tmax > t ? tmax : t;
    acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
  }
  const uint32_t tw = __builtin_amdgcn_readfirstlane(wave_max_u32(tmax));
  for (int j = 0; j < N; ++j) {
    const double4 pj = X[j];
    const uint32_t tj = __builtin_amdgcn_readfirstlane(T[j]);
    const uint32_t U = tw > tj ? tw : tj;
#pragma unroll
    for (int q = 0; q < I; ++q) {
      const double dx = pj.x - xi[q].x, dy = pj.y - xi[q].y, dz = pj.z - xi[q].z;
      const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
      double s = m_rinv3(r2, pj.w, c15, c1875);
      if (hiword(r2) <= U) {
        if (j == ii[q]) {
          s = 0.0;
        } else {
          const double4 ti = thr[ii[q]];
          const double4 tq = thr[j];
          if (close_exact(r2, ti.y, tq.y, ti.z, tq.z)) {
            s = pj.w * close_weight(r2, ti.x > tq.x ? ti.x : tq.x, f_in);
            if (count && valid[q] && j > ii[q]) ++npairs;
          }
        }
      }
      acc[q][0] = fma(s, dx, acc[q][0]);
      acc[q][1] = fma(s, dy, acc[q][1]);
      acc[q][2] = fma(s, dz, acc[q][2]);
    }
  }
}

// Kick of the whole system: v += h G a (napply times); returns this lane's m v partial sums.
template <int I, bool GROUP>
__device__ __forceinline__ void kick_system(const BatchArgs &a, int64_t o, int N, const double4 *X,
                                            const uint32_t *T, double h, int napply, bool count,
                                            double (&P)[3], unsigned &npairs) {
  const int w = GROUP ? (threadIdx.x >> 6) : 0;
  const int nw = GROUP ? kWaves : 1;
  const int nblk = (N + 64 * I - 1) / (64 * I);
  P[0] = P[1] = P[2] = 0.0;
  for (int b = w; b < nblk; b += nw) {
    double acc[I][3];
    int ii[I];
    bool valid[I];
    kick_block<I>(X, T, a.thr + o, N, b * 64 * I, a.f_in, a.c15, a.c1875, acc, ii, valid, npairs, count);
#pragma unroll
    for (int q = 0; q < I; ++q) {
      if (!valid[q]) continue;
      const double ax = a.G * acc[q][0], ay = a.G * acc[q][1], az = a.G * acc[q][2];
      double4 vi = a.v[o + ii[q]];
      for (int k = 0; k < napply; ++k) {
        vi.x = vi.x + h * ax;
        vi.y = vi.y + h * ay;
        vi.z = vi.z + h * az;
      }
      a.v[o + ii[q]] = vi;
      const double m = X[ii[q]].w;
      P[0] += m * vi.x; P[1] += m * vi.y; P[2] += m * vi.z;
    }
  }
}

template <int I, bool GROUP>
__device__ void run_system(const BatchArgs &a, int s, double4 *X, uint32_t *T, double *red) {
  const int64_t o = a.offs[s];
  const int N = (int)(a.offs[s + 1] - o);
  const int t = GROUP ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  const int nt = GROUP ? kBlock : 64;
  const double h = 0.5 * a.dt;
  const double mu = a.G * a.m0;
  for (int i = t; i < N; i += nt) {
    const double4 p = a.xm[o + i];
    const double4 th = body_thresholds(p, a.v[o + i], a.m0, a.cH, a.cV, a.n1, a.n2dt);
    a.thr[o + i] = th;
    X[i] = p;
    T[i] = hiword(th.w);
  }
  tile_sync<GROUP>();
  double P[3];
  unsigned npairs = 0;
  kick_system<I, GROUP>(a, o, N, X, T, h, 1, a.nsteps == 0 && a.npairs, P, npairs);
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
    kick_system<I, GROUP>(a, o, N, X, T, h, last ? 1 : 2, last && a.npairs, P, npairs);
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

__global__ __launch_bounds__(kBlock) void k_batched(BatchArgs a) {
  __shared__ double4 X[kMaxGroupN];
  __shared__ uint32_t T[kMaxGroupN];
  __shared__ double red[3 * kBlock];
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
    const int code = a.forced >= 0 ? a.forced : a.cfg[size_class(N)];
    if ((code & 1) && N <= kMaxWaveN) break;
    if (code & 2) run_system<2, true>(a, s, X, T, red);
    else run_system<1, true>(a, s, X, T, red);
  }
  // wave phase: wave 0 runs the system just taken, the other waves take their own
  double4 *WX = X + w * kMaxWaveN;
  uint32_t *WT = T + w * kMaxWaveN;
  int my = w == 0 ? idx : pop_wave(a.queue);
  while (my < a.nsys) {
    const int s = a.order[my];
    const int N = (int)(a.offs[s + 1] - a.offs[s]);
    const int code = a.forced >= 0 ? a.forced : a.cfg[size_class(N)];
    if (code & 2) run_system<2, false>(a, s, WX, WT, nullptr);
    else run_system<1, false>(a, s, WX, WT, nullptr);
    my = pop_wave(a.queue);
  }
}

hipError_t launch_batched(const BatchLaunch &b, hipStream_t st) {
  BatchArgs a;
  a.offs = b.offs; a.order = b.order; a.cfg = b.cfg; a.nsys = b.nsys; a.nsteps = b.nsteps;
  a.forced = b.forced; a.xm = b.xm; a.v = b.v; a.thr = b.thr; a.npairs = b.npairs; a.queue = b.queue;
  a.G = b.G; a.m0 = b.m0; a.dt = b.dt; a.f_in = b.f_in; a.cH = b.cH; a.cV = b.cV; a.n1 = b.n1;
  a.n2dt = b.n2dt; a.c15 = 1.5; a.c1875 = 1.875;
  hipError_t e = hipMemsetAsync(b.queue, 0, sizeof(unsigned), st);
  if (e != hipSuccess) return e;
  if (b.npairs) {
    e = hipMemsetAsync(b.npairs, 0, (size_t)b.nsys * sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_batched, dim3(b.grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

// Copies the bodies of m chosen systems (source offsets src, destination offsets dst[0..m]) into
// a packed scratch ensemble: one workgroup per system.
__global__ __launch_bounds__(kBlock) void k_gather(const double4 *__restrict__ xm,
                                                   const double4 *__restrict__ v,
                                                   const int64_t *__restrict__ src,
                                                   const int64_t *__restrict__ dst, int m,
                                                   double4 *__restrict__ txm,
                                                   double4 *__restrict__ tv) {
  const int k = blockIdx.x;
  if (k >= m) return;
  const int64_t s0 = src[k], d0 = dst[k], len = dst[k + 1] - dst[k];
  for (int64_t t = threadIdx.x; t < len; t += kBlock) {
    txm[d0 + t] = xm[s0 + t];
    tv[d0 + t] = v[s0 + t];
  }
}

hipError_t launch_gather(const double4 *xm, const double4 *v, const int64_t *src, const int64_t *dst,
                         int m, double4 *txm, double4 *tv, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3(m), dim3(kBlock), 0, st, xm, v, src, dst, m, txm, tv);
  return hipGetLastError();
}

int batched_max_group_n() { return kMaxGroupN; }
int batched_max_wave_n() { return kMaxWaveN; }

hipError_t batched_occupancy(int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batched, kBlock, 0);
}

}  // namespace nbk
