// Pair kernel of the H_B kick (eq. Hb) with fused close-encounter detection.
//
// Layout: one body i per lane (64 per wave, 256 per workgroup) and a j-range per workgroup row
// (blockIdx.y). All lanes of a wave visit the same j, so the j-body (x, y, z, m) and its
// threshold are wave-uniform and arrive through scalar loads into SGPRs: no LDS traffic and no
// per-lane loads inside the loop. The per-pair fast path is binary64 FMA work plus one
// quarter-rate reciprocal-square-root seed; close-encounter handling runs only for lanes whose r^2
// passes a conservative wave-level bound (one integer compare per pair).
#include "internal.hpp"

namespace nbk {
using namespace nbd;

// ------------------------------------------------------------------ pair kernel
// FORCE: accumulate accelerations; EMIT: record close partners j > i; CE: accumulate the
// complementary close-encounter acceleration; SPLIT: binary32 r^-3 core.
// perm (may be null) maps lanes to bodies. Every body's sum over j is formed in the same order
// whatever lane computes it, so the permutation changes no result bit; it only groups spatially
// close bodies into a wave, which keeps the wave-level prefilter of close pairs from firing for
// j far from all of them.
// uni (may be null) = {1, m} when every body has the same mass m: the loop then sums r^-3 d and
// multiplies by m once (one multiply less per pair), otherwise {0, 0}.
template <bool FORCE, bool EMIT, bool CE, bool SPLIT, bool UNI>
__device__ __forceinline__ void pairs_loop(const double4 *__restrict__ xm,
                                           const double4 *__restrict__ thr, double4 pi, int ii,
                                           bool valid, uint32_t tw, int j0, int j1, int n,
                                           double f_in, int *__restrict__ rowbuf, int R,
                                           double c15, double c1875, double (&a)[3],
                                           double (&ce)[3], int &nc) {
#pragma unroll 2
  for (int j = j0; j < j1; ++j) {
    const double4 pj = xm[j];
    const uint32_t tj = hiword(thr[j].w);
    const uint32_t U = tw > tj ? tw : tj;
    const double dx = pj.x - pi.x;
    const double dy = pj.y - pi.y;
    const double dz = pj.z - pi.z;
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const double mj = UNI ? 1.0 : pj.w;
    double s = 0.0;
    if (FORCE) s = SPLIT ? m_rinv3_split(r2, mj) : (UNI ? rinv3(r2, c15, c1875) : m_rinv3(r2, mj, c15, c1875));
    if (hiword(r2) <= U) {
      if (j == ii) {
        s = 0.0;
      } else {
        const double4 ti = thr[ii];
        const double4 tq = thr[j];
        if (close_exact(r2, ti.y, tq.y, ti.z, tq.z)) {
          if (FORCE) {
            const double w = close_weight(r2, ti.x > tq.x ? ti.x : tq.x, f_in);
            const double sn = UNI ? w : mj * w;
            if (CE) {
              const double ds = s - sn;
              ce[0] = fma(ds, dx, ce[0]);
              ce[1] = fma(ds, dy, ce[1]);
              ce[2] = fma(ds, dz, ce[2]);
            }
            s = sn;
          }
          if (EMIT && valid && j > ii) {
            if (nc < R) rowbuf[((size_t)blockIdx.y * R + nc) * n + ii] = j;
            ++nc;
          }
        }
      }
    }
    if (FORCE) {
      a[0] = fma(s, dx, a[0]);
      a[1] = fma(s, dy, a[1]);
      a[2] = fma(s, dz, a[2]);
    }
  }
}

template <bool FORCE, bool EMIT, bool CE, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_pairs(const double4 *__restrict__ xm,
                                                  const double4 *__restrict__ thr,
                                                  const int *__restrict__ perm,
                                                  const double2 *__restrict__ uni, int n, int chunk,
                                                  double f_in, double4 *__restrict__ part,
                                                  double4 *__restrict__ part_ce,
                                                  int *__restrict__ cnt, int *__restrict__ rowbuf,
                                                  int R, double c15, double c1875) {
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
                                             c15, c1875, a, ce, nc);
  else
    pairs_loop<FORCE, EMIT, CE, SPLIT, false>(xm, thr, pi, ii, valid, tw, j0, j1, n, f_in, rowbuf,
                                              R, c15, c1875, a, ce, nc);
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
  if (EMIT) cnt[o] = nc;
}


template <bool F, bool E, bool C, bool S>
static void go(const KickArgs &a, hipStream_t st) {
  dim3 grid(nblocks(a.n), a.nchunk);
  hipLaunchKernelGGL((k_pairs<F, E, C, S>), grid, dim3(kBlock), 0, st, a.xm, a.thr, a.perm, a.uni,
                     a.n, a.chunk, a.f_in, a.part, a.part_ce, a.cnt, a.rowbuf, a.R, 1.5, 1.875);
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
