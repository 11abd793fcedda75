// Pair kernel of the H_B kick (eq. Hb) with fused close-encounter detection.
//
// Layout: one body i per lane (64 per wave, 256 per workgroup) and a j-range per workgroup row
// (blockIdx.y). All lanes of a wave visit the same j, so the j-body (x, y, z, m) and its
// threshold are wave-uniform and arrive through scalar loads into SGPRs: no LDS traffic and no
// per-lane loads inside the loop. The per-pair fast path is binary64 FMA work plus one
// quarter-rate reciprocal-square-root seed. Close-encounter handling is reached in two
// conservative stages: a screen of 64 j at a time against the bounding box of the wave's bodies
// (a few vector instructions per 64 j), then, for the j it keeps, a per-pair integer compare.
#include "internal.hpp"

namespace nbk {
using namespace nbd;

// ------------------------------------------------------------------ pair kernel
// The close-pair part of one pair (i, j) whose j passed the block screen: the per-pair prefilter
// hi(r2) <= max(T_i, T_j), then the exact predicate, the changeover weight and the emission.
template <bool FORCE, bool EMIT, bool CE, bool UNI>
__device__ __forceinline__ void close_part(const double4 *__restrict__ thr, int ii, bool valid,
                                           uint32_t tw, int j, int n, double f_in,
                                           int *__restrict__ rowbuf, int R, double r2, double dx,
                                           double dy, double dz, double mj, double &s,
                                           double (&ce)[3], int &nc) {
  const uint32_t tj = hiword(thr[j].w);
  const uint32_t U = tw > tj ? tw : tj;
  if (hiword(r2) <= U) {
    // j taken through an empty asm statement: the compiler otherwise turns j == ii into a
    // per-lane induction variable that costs a vector add on every pair of the fast path
    int jj = j;
    asm volatile("" : "+s"(jj));
    if (jj == ii) {
      s = 0.0;
    } else {
      const double4 ti = thr[ii];
      const double4 tq = thr[j];
      if (close_exact(r2, ti.y, tq.y, ti.z, tq.z)) {
        double w;
        if (FORCE && close_weight_inner(r2, ti.x > tq.x ? ti.x : tq.x, f_in, w)) {
          const double sn = UNI ? w : mj * w;
          if (CE) {
            const double ds = s - sn;
            ce[0] = fma(ds, dx, ce[0]);
            ce[1] = fma(ds, dy, ce[1]);
            ce[2] = fma(ds, dz, ce[2]);
          }
          s = sn;
        }
        if (EMIT && valid && jj > ii) {
          if (nc < R) rowbuf[((size_t)blockIdx.y * R + nc) * n + ii] = jj;
          ++nc;
        }
      }
    }
  }
}

// r^-3 (times m_j unless all masses are equal) of one pair, and the offsets it multiplies.
template <bool SPLIT, bool UNI>
__device__ __forceinline__ double pair_weight(const double4 &pi, const double4 &pj, double c15,
                                              double &dx, double &dy, double &dz, double &r2) {
  dx = pj.x - pi.x;
  dy = pj.y - pi.y;
  dz = pj.z - pi.z;
  r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  return SPLIT ? m_rinv3_split(r2, UNI ? 1.0 : pj.w)
               : (UNI ? rinv3(r2, c15) : m_rinv3(r2, pj.w, c15));
}

// One pair of a j-block with no close pair: the fast path alone.
template <bool SPLIT, bool UNI>
__device__ __forceinline__ void pair_far(const double4 &pi, const double4 &pj, double c15,
                                         double (&a)[3]) {
  double dx, dy, dz, r2;
  const double s = pair_weight<SPLIT, UNI>(pi, pj, c15, dx, dy, dz, r2);
  a[0] = fma(s, dx, a[0]);
  a[1] = fma(s, dy, a[1]);
  a[2] = fma(s, dz, a[2]);
}

// A block of LEN j-bodies with no pair near enough to need the predicate. No per-j branch; the
// j-bodies alternate between two pairs of scalar registers, each pair loaded one step ahead of
// its use (the last step reloads bodies LEN - 2 and LEN - 1, unused).
template <bool SPLIT, bool UNI, int LEN>
__device__ __forceinline__ void far_block(const double4 *__restrict__ xb, const double4 &pi,
                                          double c15, double (&a)[3]) {
  double4 c0 = xb[0], c1 = xb[1];
  for (int k = 0; k < LEN; k += 4) {
    const double4 n0 = xb[k + 2], n1 = xb[k + 3];
    pair_far<SPLIT, UNI>(pi, c0, c15, a);
    pair_far<SPLIT, UNI>(pi, c1, c15, a);
    const int kk = min(k + 4, LEN - 2);
    c0 = xb[kk];
    c1 = xb[kk + 1];
    pair_far<SPLIT, UNI>(pi, n0, c15, a);
    pair_far<SPLIT, UNI>(pi, n1, c15, a);
  }
}

// One pair of the force loop: r^-3 on the fast path; close_part only for a screened-in j.
template <bool EMIT, bool CE, bool SPLIT, bool UNI>
__device__ __forceinline__ void pair_force(const double4 *__restrict__ thr, const double4 &pi,
                                           const double4 &pj, int ii, bool valid, uint32_t tw, int j,
                                           int n, double f_in, int *__restrict__ rowbuf, int R,
                                           double c15, bool screened, double (&a)[3],
                                           double (&ce)[3], int &nc) {
  double dx, dy, dz, r2;
  double s = pair_weight<SPLIT, UNI>(pi, pj, c15, dx, dy, dz, r2);
  if (screened)
    close_part<true, EMIT, CE, UNI>(thr, ii, valid, tw, j, n, f_in, rowbuf, R, r2, dx, dy, dz,
                                    UNI ? 1.0 : pj.w, s, ce, nc);
  a[0] = fma(s, dx, a[0]);
  a[1] = fma(s, dy, a[1]);
  a[2] = fma(s, dz, a[2]);
}

// FORCE: accumulate accelerations; EMIT: record close partners j > i; CE: accumulate the
// complementary close-encounter acceleration; SPLIT: binary32 r^-3 core.
// perm (may be null) maps lanes to bodies. Every body's sum over j is formed in the same order
// whatever lane computes it, so the permutation changes no result bit; it only groups spatially
// close bodies into a wave, which keeps the bounding box of the wave small and the screen below
// selective.
// uni (may be null) = {1, m} when every body has the same mass m: the loop then sums r^-3 d and
// multiplies by m once (one multiply less per pair), otherwise {0, 0}.
//
// Block screen: the j-range is taken 64 bodies at a time; lane l tests j = jb + l against the
// bounding box of the wave's 64 i-bodies. If even the box distance d2 has hi(d2) >= U_j + 2, no
// pair (i, j) of the wave can pass the per-pair prefilter: the computed r2 of any such pair is at
// least d2 up to a few ulp, and one unit of the high word is a relative 2^-20. Those j run the
// fast path only; the ballot of the others selects, per j, the uniform branch into close_part.
// The arithmetic of every pair is the same on both paths, so the screen changes no result bit.
template <bool FORCE, bool EMIT, bool CE, bool SPLIT, bool UNI>
__device__ __forceinline__ void pairs_loop(const double4 *__restrict__ xm,
                                           const double4 *__restrict__ thr, double4 pi, int ii,
                                           bool valid, uint32_t tw, int j0, int j1, int n,
                                           double f_in, int *__restrict__ rowbuf, int R,
                                           double c15, double (&a)[3],
                                           double (&ce)[3], int &nc) {
  const int lane = threadIdx.x & 63;
  // lanes past n hold body n - 1, a real body: the box stays conservative
  const double bx0 = wave_min_f64(pi.x), bx1 = wave_max_f64(pi.x);
  const double by0 = wave_min_f64(pi.y), by1 = wave_max_f64(pi.y);
  const double bz0 = wave_min_f64(pi.z), bz1 = wave_max_f64(pi.z);
  // 1.5 held in a VGPR for the whole loop: one VOP3 instruction reads at most one scalar operand,
  // and the j-body's coordinates arrive in SGPRs
  double c15v;
  asm volatile("v_mov_b64 %0, %1" : "=v"(c15v) : "s"(c15));
  for (int jb = j0; jb < j1; jb += 64) {
    const int jl = jb + lane;
    bool near = false;
    if (jl < j1) {
      const double4 q = xm[jl];
      const uint32_t tq = hiword(thr[jl].w);
      const uint32_t U = tw > tq ? tw : tq;
      const double ex = fmax(fmax(bx0 - q.x, q.x - bx1), 0.0);
      const double ey = fmax(fmax(by0 - q.y, q.y - by1), 0.0);
      const double ez = fmax(fmax(bz0 - q.z, q.z - bz1), 0.0);
      const double d2 = fma(ez, ez, fma(ey, ey, ex * ex));
      near = !(hiword(d2) >= U + 2u);
    }
    const unsigned long long mask = __ballot(near);
    const int je = min(j1, jb + 64);
    if (!FORCE) {
      // without forces only the screened-in j need a visit
      unsigned long long m = mask;
      while (m) {
        const int j = jb + __builtin_ctzll(m);
        m &= m - 1;
        const double4 pj = xm[j];
        const double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        double s = 0.0;
        close_part<FORCE, EMIT, CE, UNI>(thr, ii, valid, tw, j, n, f_in, rowbuf, R, r2, dx, dy, dz,
                                         1.0, s, ce, nc);
      }
      continue;
    }
    if (mask == 0 && je - jb == 64) {
      // the common case: a whole block with no pair near enough to need the predicate
      far_block<SPLIT, UNI, 64>(xm + jb, pi, c15v, a);
      continue;
    }
    if (mask == 0 && je - jb == 32) {
      // the half blocks of the chunks of small systems
      far_block<SPLIT, UNI, 32>(xm + jb, pi, c15v, a);
      continue;
    }
    // a block with screened-in j (or a partial block): j-bodies two at a time, the scalar loads
    // of the next two issued before the arithmetic of the current two
    int j = jb;
    if (j + 2 <= je) {
      double4 c0 = xm[j], c1 = xm[j + 1];
      for (; j + 4 <= je; j += 2) {
        const double4 n0 = xm[j + 2], n1 = xm[j + 3];
        pair_force<EMIT, CE, SPLIT, UNI>(thr, pi, c0, ii, valid, tw, j, n, f_in, rowbuf, R, c15v,
                                         (mask >> (j - jb)) & 1ull, a, ce, nc);
        pair_force<EMIT, CE, SPLIT, UNI>(thr, pi, c1, ii, valid, tw, j + 1, n, f_in, rowbuf, R, c15v,
                                         (mask >> (j + 1 - jb)) & 1ull, a, ce, nc);
        c0 = n0;
        c1 = n1;
      }
      pair_force<EMIT, CE, SPLIT, UNI>(thr, pi, c0, ii, valid, tw, j, n, f_in, rowbuf, R, c15v,
                                       (mask >> (j - jb)) & 1ull, a, ce, nc);
      pair_force<EMIT, CE, SPLIT, UNI>(thr, pi, c1, ii, valid, tw, j + 1, n, f_in, rowbuf, R, c15v,
                                       (mask >> (j + 1 - jb)) & 1ull, a, ce, nc);
      j += 2;
    }
    for (; j < je; ++j)
      pair_force<EMIT, CE, SPLIT, UNI>(thr, pi, xm[j], ii, valid, tw, j, n, f_in, rowbuf, R, c15v,
                                       (mask >> (j - jb)) & 1ull, a, ce, nc);
  }
}

// The kernel body: one lane per body i of the launch's rows, the j-range of blockIdx.y.
template <bool FORCE, bool EMIT, bool CE, bool SPLIT>
__device__ __forceinline__ void pairs_body(const double4 *__restrict__ xm,
                                           const double4 *__restrict__ thr,
                                           const int *__restrict__ perm,
                                           const double2 *__restrict__ uni, int n, int chunk,
                                           double f_in, double4 *__restrict__ part,
                                           double4 *__restrict__ part_ce, int *__restrict__ cnt,
                                           int *__restrict__ rowbuf, int R, double c15,
                                           int *__restrict__ rowsum,
                                           unsigned long long *__restrict__ rowmask) {
  const int lane_body = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = lane_body < n;
  const int lb = valid ? lane_body : n - 1;
  const int ii = perm ? perm[lb] : lb;
  const double4 pi = xm[ii];
  // wave-uniform prefilter bound: a pair (i, j) can be close only if r^2 <= max(T_i, T_j)
  const uint32_t tw = __builtin_amdgcn_readfirstlane(wave_max_u32(hiword(thr[ii].w)));
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  double a[3] = {0.0, 0.0, 0.0};
  double ce[3] = {0.0, 0.0, 0.0};
  int nc = 0;
  double mu = 1.0;
  bool uniform = false;
  if (FORCE && uni) {
    const double2 u = uni[0];
    uniform = u.x != 0.0;
    mu = u.y;
  }
  if (uniform)
    pairs_loop<FORCE, EMIT, CE, SPLIT, true>(xm, thr, pi, ii, valid, tw, j0, j1, n, f_in, rowbuf, R,
                                             c15, a, ce, nc);
  else
    pairs_loop<FORCE, EMIT, CE, SPLIT, false>(xm, thr, pi, ii, valid, tw, j0, j1, n, f_in, rowbuf,
                                              R, c15, a, ce, nc);
  if (!valid) return;
  const size_t o = (size_t)blockIdx.y * n + ii;
  if (FORCE) {
    if (uniform) { a[0] *= mu; a[1] *= mu; a[2] *= mu; }
    part[o] = make_double4(a[0], a[1], a[2], 0.0);
  }
  if (CE) {
    if (uniform) { ce[0] *= mu; ce[1] *= mu; ce[2] *= mu; }
    part_ce[o] = make_double4(ce[0], ce[1], ce[2], 0.0);
  }
  if (EMIT) {
    cnt[o] = nc;
    if (nc > 0 && rowsum) {
      atomicAdd(rowsum + ii, nc);
      atomicOr(rowmask + (size_t)ii * kRowMaskWords + (blockIdx.y >> 6), 1ull << (blockIdx.y & 63));
    }
  }
}

// Register budget of the kernels without the close-encounter part: 80 VGPRs (six waves per SIMD
// in the compiler's model), no spills. Measured resident waves per SIMD on the 32768 disk: 4.1 at
// 86 VGPRs, 4.9 at 80, 5.6 at 72 and 6.3 at 64 (the last two with spills outside the fast loop),
// VALU busy 0.88-0.90 in every case: the issue efficiency of this instruction mix does not rise
// with occupancy beyond five waves. The kernels with the close-encounter part keep five waves in
// the compiler's model, where they do not spill.
template <bool FORCE, bool EMIT, bool SPLIT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_pairs(
    const double4 *__restrict__ xm, const double4 *__restrict__ thr, const int *__restrict__ perm,
    const double2 *__restrict__ uni, int n, int chunk, double f_in, double4 *__restrict__ part,
    double4 *__restrict__ part_ce, int *__restrict__ cnt, int *__restrict__ rowbuf, int R,
    double c15, int *__restrict__ rowsum, unsigned long long *__restrict__ rowmask) {
  pairs_body<FORCE, EMIT, false, SPLIT>(xm, thr, perm, uni, n, chunk, f_in, part, part_ce, cnt,
                                        rowbuf, R, c15, rowsum, rowmask);
}

template <bool EMIT, bool SPLIT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_pairs_ce(
    const double4 *__restrict__ xm, const double4 *__restrict__ thr, const int *__restrict__ perm,
    const double2 *__restrict__ uni, int n, int chunk, double f_in, double4 *__restrict__ part,
    double4 *__restrict__ part_ce, int *__restrict__ cnt, int *__restrict__ rowbuf, int R,
    double c15, int *__restrict__ rowsum, unsigned long long *__restrict__ rowmask) {
  pairs_body<true, EMIT, true, SPLIT>(xm, thr, perm, uni, n, chunk, f_in, part, part_ce, cnt,
                                      rowbuf, R, c15, rowsum, rowmask);
}

template <bool F, bool E, bool C, bool S>
static void go(const KickArgs &a, hipStream_t st) {
  dim3 grid(nblocks(a.n), a.nchunk);
  if constexpr (C)
    hipLaunchKernelGGL((k_pairs_ce<E, S>), grid, dim3(kBlock), 0, st, a.xm, a.thr, a.perm, a.uni, a.n,
                       a.chunk, a.f_in, a.part, a.part_ce, a.cnt, a.rowbuf, a.R, 1.5,
                       E ? a.rowsum : nullptr, E ? a.rowmask : nullptr);
  else
    hipLaunchKernelGGL((k_pairs<F, E, S>), grid, dim3(kBlock), 0, st, a.xm, a.thr, a.perm, a.uni, a.n,
                       a.chunk, a.f_in, a.part, a.part_ce, a.cnt, a.rowbuf, a.R, 1.5,
                       E ? a.rowsum : nullptr, E ? a.rowmask : nullptr);
}

hipError_t launch_pairs(const KickArgs &a, bool force, bool emit, bool ce, bool split,
                        hipStream_t st) {
  if (!force) {
    go<false, true, false, false>(a, st);
  } else if (split) {
    if (emit) { ce ? go<true, true, true, true>(a, st) : go<true, true, false, true>(a, st); }
    else { ce ? go<true, false, true, true>(a, st) : go<true, false, false, true>(a, st); }
  } else {
    if (emit) { ce ? go<true, true, true, false>(a, st) : go<true, true, false, false>(a, st); }
    else { ce ? go<true, false, true, false>(a, st) : go<true, false, false, false>(a, st); }
  }
  return hipGetLastError();
}

}  // namespace nbk
