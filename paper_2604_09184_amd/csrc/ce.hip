// Close-encounter drift: the H_A part of the step (eq. Ha) in full, including the [1 - K] pair
// term, for the bodies of close-encounter groups; bodies in no group keep the Kepler drift.
//
// Within a group the equations of motion are
//   dx_i/dt = v_i,
//   dv_i/dt = -G m0 x_i/|x_i|^3 + G sum_{j in group, j != i} m_j ((1 - K)/r^3 + K'(r)/r^2) d_ij,
// d_ij = x_j - x_i: minus the gradient of the [1 - K] part of the pair potential, which vanishes
// for r >= rc_ij. They are integrated with the Gragg-Bulirsch-Stoer method: modified-midpoint
// sweeps with 2, 4, ..., 10 substeps over a macro step H, extrapolated to zero substep length as a
// polynomial in (H/n)^2 (Aitken-Neville); a macro step is accepted when the last two extrapolants
// agree to the tolerance relative to the group's largest position and velocity, and halved
// otherwise. With intermediate changeover levels the [1 - K] factor becomes the product of the
// levels' [1 - K_l]; with collisions, members in contact merge (see k_ce_drift).
//
// One workgroup of four waves per group of at most 64 bodies (the work layout is described at the
// integrator below): the positions of other members arrive by lane shuffles, every step-size
// decision is taken on wave-wide reductions of identical data in every wave, so the integration is
// uniform across the workgroup and deterministic. The launch holds only resident workgroups; they
// take groups from a queue until the device-side group count is exhausted.
#include "internal.hpp"
#include "kepler_core.hpp"

#include <algorithm>

namespace nbk {
using namespace nbd;

// ------------------------------------------------------------------ group member lists
// Group sizes from caller-given labels (every body labelled with the smallest index of its group).
__global__ __launch_bounds__(kBlock) void k_gzero(int n, int *__restrict__ gsize,
                                                  int *__restrict__ gfill, int *__restrict__ counter) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    gsize[i] = 0;
    gfill[i] = 0;
  }
  if (i < kGroupCounters) counter[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_gcount(const int *__restrict__ label, int n,
                                                   int *__restrict__ gsize) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) atomicAdd(gsize + label[i], 1);
}

// in[i] = 1 for a body that shares its group with another body; slices of the member array by
// atomic allocation (counter[1]) and the roots of the groups into a list (counter[0]): where a
// group's slice sits does not matter, each group is integrated on its own with its members ordered
// by body index.
__global__ __launch_bounds__(kBlock) void k_galloc(const int *__restrict__ label,
                                                   const int *__restrict__ gsize, int n,
                                                   int *__restrict__ in, int *__restrict__ gstart,
                                                   int *__restrict__ groot, int *__restrict__ counter,
                                                   const int *__restrict__ deg,
                                                   int *__restrict__ skip) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const bool member = gsize[label[i]] >= 2;
  in[i] = member;
  if (skip) skip[i] = !(deg[i] > 0 && !member);
  if (label[i] == i && gsize[i] >= 2) {
    gstart[i] = atomicAdd(counter + 1, gsize[i]);
    groot[atomicAdd(counter, 1)] = i;
  }
}

// Members into their group's slots (slot order is arbitrary; the integrator orders them by body
// index).
__global__ __launch_bounds__(kBlock) void k_gfill(const int *__restrict__ label,
                                                  const int *__restrict__ in, int n,
                                                  const int *__restrict__ gstart,
                                                  int *__restrict__ gfill, int *__restrict__ gmem) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || !in[i]) return;
  const int r = label[i];
  gmem[gstart[r] + atomicAdd(gfill + r, 1)] = i;
}

// ------------------------------------------------------------------ integrator
// Work layout. A group of k <= 64 bodies is integrated by one workgroup of kCeWaves = 4 waves.
// A macro step extrapolates kCols = 5 modified-midpoint sweeps (n = 2, 4, ..., 10 substeps; a
// sweep costs n evaluations of the right-hand side after the f(y) it starts from, plus one for
// the smoothing). The sweeps are independent of one another, so waves 0, 1 and 3 run the sweeps
// n = 10, 8 and 4 and wave 2 the sweeps n = 6 and 2 (f(y) shared): 11, 9, 9 and 5 evaluations, 11
// on the longest path against 31 for all five in a row. Their end values meet in LDS, and every
// wave then forms the same extrapolation tableau, takes the same decision and updates the same
// state, so the waves stay in step without further exchange.
//
// Five columns rather than eight (n up to 16, 19 evaluations on the longest path with the same
// pairing): the extrapolation order is lower, so a macro step is shorter and more of them are
// needed, but each costs 11 instead of 19 evaluations, and the drift's length is that of its
// slowest group's chain of macro steps. On the 2048- and 32768-body disks the slowest group then
// takes 20-25 % more macro steps for a 40 % cheaper step.
//
// Within a wave, body slot s (0 <= s < k) sits on the P lanes s P + r, r = 0 .. P - 1, with
// P = min(kp, 64/kp) and kp the power of two at or above k: replica r sums the pair terms of every
// P-th member, and the replicas' partial sums meet in a butterfly inside a 16-lane row made of DPP
// moves (lane exchanges xor 1 and xor 2, then the half-row and row mirrors), each stage an addition
// of two equal-sized partial sums in either order, so every replica ends with the same bits. A group
// of up to 8 bodies thus needs one pair term per replica and log2(kp) butterfly stages.
constexpr int kCeWaves = 4;
constexpr int kCols = 5;
constexpr int kMaxMacroSteps = 20000;
constexpr int kMaxBisections = 80;       // contact-time bisection: at most 80 halvings of a step
constexpr double kParkRadius = 1e6;      // orbit radius of bodies merged away

// Largest value over the wave, uniform: DPP maxima inside each 16-lane row, then the four rows
// through scalar registers.
__device__ __forceinline__ double wave_max_d(double x) {
  x = fmax(x, dpp_f64<0xB1>(x));
  x = fmax(x, dpp_f64<0x4E>(x));
  x = fmax(x, dpp_f64<0x141>(x));
  x = fmax(x, dpp_f64<0x140>(x));
  const long long b = __double_as_longlong(x);
  double m = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, 16 * r);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), 16 * r);
    const double q = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    m = r == 0 ? q : fmax(m, q);
  }
  return m;
}

// Per-member values in ascending body order: G m, rc, 1/((1 - f_in) rc) and the contact radius
// f R (G m and f R change when members merge).
struct CeMember {
  double Gm, rc, ispan, fR;
};

// Shared state of one group's integration (LDS): the tableau's end values (double buffered), the
// slot of each member rank, the member values, masses, radii and body indices by rank, and the
// critical radii rc_l and 1/((1 - f_in) rc_l) of the changeover levels by rank.
struct CeShared {
  double est[2][kCols][6][64];
  CeMember mem[64];
  double mass[64], rad[64];
  double lrc[kMaxLevels][64], lisp[kMaxLevels][64];
  int owner[64], body[64];
};

// Per-lane constants of one group's integration (nl: changeover levels weighting the pair term).
struct CeLane {
  int k, iters, P, rep, slot, wv, rank, nl;
  bool act;
  double rc, ispan, Gm0, f_in, tol;
};

// A lane's partners: for iteration it the member q = rep + it P (in ascending body order), the lane
// src of its first replica, and whether the term counts (a member, and not the lane's own body).
struct CePartner {
  int src, q;
  bool use;
  CeMember m;
  // the pair's critical radius max(rc_i, rc_j) and 1/((1 - f_in) rc_ij) of the step's level, and
  // of the first intermediate level when there is one
  double rcij, isp, rcij1, isp1;
};

__device__ __forceinline__ CePartner ce_partner(int q, const CeLane &L, const CeShared &sh) {
  const bool valid = q < L.k;
  const int qq = valid ? q : 0;
  CePartner p;
  p.q = qq;
  p.src = sh.owner[qq] * L.P;
  p.use = L.act && valid && sh.owner[qq] != L.slot;
  p.m = sh.mem[qq];
  const bool mine = L.rc > p.m.rc;
  p.rcij = mine ? L.rc : p.m.rc;
  p.isp = mine ? L.ispan : p.m.ispan;
  p.rcij1 = p.rcij;
  p.isp1 = p.isp;
  if (L.nl >= 2) {
    const double ri = sh.lrc[1][L.rank], rj = sh.lrc[1][qq];
    const bool mine1 = ri > rj;
    p.rcij1 = mine1 ? ri : rj;
    p.isp1 = mine1 ? sh.lisp[1][L.rank] : sh.lisp[1][qq];
  }
  return p;
}

// Pair term of one partner, added to a. The coefficient is G m_j ((1 - K)/r^3 + K'(r)/r^2); with y
// the changeover variable clamped to [0, 1] and D = 2y^2 - 2y + 1, 1 - K = (1 - y)^2/D and
// K'(r) = 2y(1 - y)/(D^2 (1 - f_in) rc_ij), which gives 1/r^3 inside f_in rc_ij and 0 beyond rc_ij
// with no branch. No division or square root: r^-1 and 1/D come from refined hardware estimates.
//
// With intermediate changeover levels the pair potential is weighted by W = prod_l [1 - K_l] (one
// factor per level, each with its own rc_l), and the coefficient is G m_j (W/r^3 - W'(r)/r^2).
template <int NL>
__device__ __forceinline__ void ce_pair(const double (&z)[6], const CePartner &p, const CeLane &L,
                                        const CeShared &sh, double &a0, double &a1, double &a2) {
  // a term that does not count (no member, or the lane's own body) is moved 1e30 away along x:
  // there the changeover weight is exactly zero, so the term adds exactly zero (times finite
  // offsets) with no branch. The exchange runs on every lane (a lane shuffle reads only from
  // active lanes), and the offset is added to its result
  const double off = p.use ? 0.0 : 1e30;
  const double dx = (__shfl(z[0], p.src, 64) - z[0]) + off;
  const double dy = __shfl(z[1], p.src, 64) - z[1];
  const double dz = __shfl(z[2], p.src, 64) - z[2];
  // (the library builds with contraction off: products that feed a sum are fused explicitly)
  const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  const double ir = rinv_refined(r2);
  const double r = r2 * ir;
  const double f_in = L.f_in;
  double c;
  if (NL == 1) {
    const double rcij = p.rcij, isp = p.isp;
    const double y = fmin(fmax(fma(-f_in, rcij, r) * isp, 0.0), 1.0);
    const double omy = 1.0 - y, y2 = 2.0 * y;
    const double iD = recip_refined(fma(y2, y - 1.0, 1.0));
    const double u = omy * iD;
    // (1 - K) ir + K', times ir^2
    c = (ir * ir) * fma(u * omy, ir, ((y2 * u) * iD) * isp);
  } else if (NL == 2) {
    // W = [1 - K_0][1 - K_1], the two levels' constants kept with the partner
    double W = 1.0, dW = 0.0;
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const double rcij = l == 0 ? p.rcij : p.rcij1;
      const double isp = l == 0 ? p.isp : p.isp1;
      const double y = fmin(fmax(fma(-f_in, rcij, r) * isp, 0.0), 1.0);
      const double omy = 1.0 - y, y2 = 2.0 * y;
      const double iD = recip_refined(fma(y2, y - 1.0, 1.0));
      const double u = omy * iD;
      const double omK = u * omy, dK = ((y2 * u) * iD) * isp;
      dW = fma(dW, omK, -(W * dK));
      W = W * omK;
    }
    c = (ir * ir) * fma(W, ir, -dW);
  } else {
    double W = 1.0, dW = 0.0;
    for (int l = 0; l < L.nl; ++l) {
      const double rci = sh.lrc[l][L.rank], rcj = sh.lrc[l][p.q];
      const bool mine = rci > rcj;
      const double rcij = mine ? rci : rcj;
      const double isp = mine ? sh.lisp[l][L.rank] : sh.lisp[l][p.q];
      const double y = fmin(fmax(fma(-f_in, rcij, r) * isp, 0.0), 1.0);
      const double omy = 1.0 - y, y2 = 2.0 * y;
      const double iD = recip_refined(fma(y2, y - 1.0, 1.0));
      const double u = omy * iD;
      const double omK = u * omy, dK = ((y2 * u) * iD) * isp;
      dW = fma(dW, omK, -(W * dK));
      W = W * omK;
    }
    c = (ir * ir) * fma(W, ir, -dW);
  }
  const double cm = c * p.m.Gm;
  a0 = fma(cm, dx, a0);
  a1 = fma(cm, dy, a1);
  a2 = fma(cm, dz, a2);
}


template <int CTRL>
__device__ __forceinline__ void ce_row_add(double &a0, double &a1, double &a2) {
  a0 += dpp_f64<CTRL>(a0);
  a1 += dpp_f64<CTRL>(a1);
  a2 += dpp_f64<CTRL>(a2);
}

// Partners of a lane kept in registers; members beyond them are read from LDS.
constexpr int kCeRegPartners = 4;

// f = (v, a) of this lane's body at the state z. PT > 0: P = PT replicas and one partner per
// replica (groups of up to 8 bodies), known at compile time; PT = 0: P and the partner count from L.
template <int NL, int PT>
__device__ __forceinline__ void ce_rhs(const double (&z)[6], const CeLane &L, const CeShared &sh,
                                       const CePartner (&pr)[kCeRegPartners], bool alive,
                                       double (&f)[6]) {
  const int P = PT > 0 ? PT : L.P;
  // the central term first: it does not depend on the partners, so its latency overlaps their
  // exchange
  const double r2 = fma(z[2], z[2], fma(z[1], z[1], z[0] * z[0]));
  const double ir = rinv_refined(r2);
  const double s = -L.Gm0 * (ir * ir * ir);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (PT > 0 || L.iters == 1) {
    ce_pair<NL>(z, pr[0], L, sh, a0, a1, a2);
  } else {
    // independent terms side by side (masked beyond the members)
#pragma unroll
    for (int u = 0; u < kCeRegPartners; ++u) ce_pair<NL>(z, pr[u], L, sh, a0, a1, a2);
    for (int it = kCeRegPartners; it < L.iters; it += kCeRegPartners) {
#pragma unroll
      for (int u = 0; u < kCeRegPartners; ++u) {
        const CePartner p = ce_partner(L.rep + (it + u) * P, L, sh);
        ce_pair<NL>(z, p, L, sh, a0, a1, a2);
      }
    }
  }
  if (P >= 2) ce_row_add<0xB1>(a0, a1, a2);    // quad_perm [1, 0, 3, 2]: lane xor 1
  if (P >= 4) ce_row_add<0x4E>(a0, a1, a2);    // quad_perm [2, 3, 0, 1]: lane xor 2
  if (P >= 8) ce_row_add<0x141>(a0, a1, a2);   // half-row mirror: lane i <-> 7 - i
  if (P >= 16) ce_row_add<0x140>(a0, a1, a2);  // row mirror: lane i <-> 15 - i
  // a body merged away is held fixed
  f[0] = alive ? z[3] : 0.0;
  f[1] = alive ? z[4] : 0.0;
  f[2] = alive ? z[5] : 0.0;
  f[3] = alive ? fma(s, z[0], a0) : 0.0;
  f[4] = alive ? fma(s, z[1], a1) : 0.0;
  f[5] = alive ? fma(s, z[2], a2) : 0.0;
}

// Modified-midpoint sweep of ns substeps over H from y, with f0 = f(y): the end value
// (z_n + z_{n-1} + hs f(z_n))/2.
template <int NL, int PT>
__device__ __forceinline__ void ce_sweep(const double (&y)[6], const double (&f0)[6], double H, int ns,
                                         const CeLane &L, const CeShared &sh,
                                         const CePartner (&pr)[kCeRegPartners], bool alive,
                                         double (&est)[6]) {
  const double hs = H / ns;
  double zm[6], zc[6], f[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    zm[i] = y[i];
    zc[i] = fma(hs, f0[i], y[i]);
  }
  // z_{m+1} = z_{m-1} + 2 hs f(z_m), m = 1 .. ns - 1, two steps per iteration so that the two state
  // arrays trade roles without copies (ns is even: one step is left over at the end)
  const double h2 = 2.0 * hs;
  for (int s = 1; s + 1 < ns; s += 2) {
    ce_rhs<NL, PT>(zc, L, sh, pr, alive, f);
#pragma unroll
    for (int i = 0; i < 6; ++i) zm[i] = fma(h2, f[i], zm[i]);
    ce_rhs<NL, PT>(zm, L, sh, pr, alive, f);
#pragma unroll
    for (int i = 0; i < 6; ++i) zc[i] = fma(h2, f[i], zc[i]);
  }
  ce_rhs<NL, PT>(zc, L, sh, pr, alive, f);
#pragma unroll
  for (int i = 0; i < 6; ++i) zm[i] = fma(h2, f[i], zm[i]);
  // now zm = z_ns and zc = z_{ns-1}
  ce_rhs<NL, PT>(zm, L, sh, pr, alive, f);
#pragma unroll
  for (int i = 0; i < 6; ++i) est[i] = 0.5 * fma(hs, f[i], zm[i] + zc[i]);
}

// Aitken-Neville over the kCols sweeps (substep counts 2c + 2) of one component:
// T[c][0] = e[c], T[c][j] = T[c][j-1] + (T[c][j-1] - T[c-1][j-1]) / ((n_c/n_{c-j})^2 - 1).
// Returns T[want][want] and, in err[c], max(err[c], |T[c][c] - T[c][c-1]| iscale) for c >= 2.
__device__ __forceinline__ double ce_tableau(const double (&e)[kCols], double iscale, int want,
                                             double (&err)[kCols]) {
  double prev[kCols], cur[kCols], out = e[0];
#pragma unroll
  for (int c = 0; c < kCols; ++c) {
    cur[0] = e[c];
#pragma unroll
    for (int j = 1; j <= c; ++j) {
      // 1/((n_c/n_{c-j})^2 - 1) is a constant once the loops are unrolled: a multiplication
      const double ratio = (double)(c + 1) / (double)(c + 1 - j);
      cur[j] = fma(cur[j - 1] - prev[j - 1], 1.0 / (ratio * ratio - 1.0), cur[j - 1]);
    }
    if (c >= 2) err[c] = fmax(err[c], fabs(cur[c] - cur[c - 1]) * iscale);
    if (c == want) out = cur[c];
#pragma unroll
    for (int j = 0; j <= c; ++j) prev[j] = cur[j];
  }
  return out;
}

// One macro-step attempt over H from y (all four waves together): returns the accepted column
// (identical in every wave) or -1; y1 receives the accepted extrapolant.
template <int NL, int PT>
__device__ __forceinline__ int ce_attempt(const double (&y)[6], double H, bool alive, const CeLane &L,
                                          CeShared &sh, const CePartner (&pr)[kCeRegPartners],
                                          int &buf, double (&y1)[6]) {
  const bool live = L.act && alive;
  const double sx = wave_max_d(live ? fmax(fabs(y[0]), fmax(fabs(y[1]), fabs(y[2]))) : 0.0);
  const double sv = wave_max_d(live ? fmax(fabs(y[3]), fmax(fabs(y[4]), fabs(y[5]))) : 0.0);
  const double isx = 1.0 / sx, isv = 1.0 / sv;
  // f(y) starts every sweep of the wave: evaluated once
  double f0[6];
  ce_rhs<NL, PT>(y, L, sh, pr, alive, f0);
  // the wave's columns: kCols - 1 - w, and column 0 for wave 2 (wave-uniform)
  static_assert(kCols == 5 && kCeWaves == 4, "the column split below is for 5 columns on 4 waves");
#pragma unroll
  for (int cc = 0; cc < 2; ++cc) {
    const int c = cc == 0 ? kCols - 1 - L.wv : (L.wv == 2 ? 0 : -1);
    if (c < 0) continue;
    double est[6];
    ce_sweep<NL, PT>(y, f0, H, 2 * c + 2, L, sh, pr, alive, est);
    if (L.rep == 0)
#pragma unroll
      for (int i = 0; i < 6; ++i) sh.est[buf][c][i][L.slot] = est[i];
  }
  __syncthreads();
  // tableau of every component; the first pass finds the accepted column
  double err[kCols] = {};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double e[kCols];
#pragma unroll
    for (int c = 0; c < kCols; ++c) e[c] = sh.est[buf][c][i][L.slot];
    (void)ce_tableau(e, i < 3 ? isx : isv, -1, err);
  }
  int accepted = -1;
#pragma unroll
  for (int c = 2; c < kCols; ++c)
    if (accepted < 0 && __ballot(live && !(err[c] <= L.tol)) == 0) accepted = c;
  if (accepted >= 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double e[kCols], dummy[kCols] = {};
#pragma unroll
      for (int c = 0; c < kCols; ++c) e[c] = sh.est[buf][c][i][L.slot];
      y1[i] = ce_tableau(e, 1.0, accepted, dummy);
    }
  }
  buf ^= 1;
  return accepted;
}

// Lowest (rank_lo, rank_hi) pair of live members closer than f (R_lo + R_hi) at the state y, as
// rank_lo * 64 + rank_hi, or -1; identical in every lane and wave.
__device__ __forceinline__ void ce_contact_test(const double (&y)[6], double fR, const CeLane &L,
                                                const CePartner &p, int &key) {
  const double dx = __shfl(y[0], p.src, 64) - y[0];
  const double dy = __shfl(y[1], p.src, 64) - y[1];
  const double dz = __shfl(y[2], p.src, 64) - y[2];
  const double lim = fR + p.m.fR;
  if (p.use && fR > 0.0 && p.m.fR > 0.0 && dx * dx + dy * dy + dz * dz < lim * lim) {
    const int lo = min(L.rank, p.q), hi = max(L.rank, p.q);
    key = min(key, lo * 64 + hi);
  }
}

__device__ __forceinline__ int ce_contact(const double (&y)[6], double fR, const CeLane &L,
                                          const CeShared &sh, const CePartner (&pr)[kCeRegPartners]) {
  int key = 0x7fffffff;
#pragma unroll
  for (int u = 0; u < kCeRegPartners; ++u)
    if (u < L.iters) ce_contact_test(y, fR, L, pr[u], key);
  for (int it = kCeRegPartners; it < L.iters; ++it)
    ce_contact_test(y, fR, L, ce_partner(L.rep + it * L.P, L, sh), key);
  if (__ballot(key != 0x7fffffff) == 0) return -1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) key = min(key, __shfl_xor(key, o, 64));
  return key;
}

// Adaptive integration of y over the time Ltot (macro steps from H = Ltot; halved when rejected,
// 2.5 H after acceptance at column <= 2, 1.5 H at column 3, 1.2 H at column 4). With
// check, every accepted step is followed by a contact test and the integration stops at the
// first step that ends in contact: y then holds that step's start, done the time covered before
// it and Hc its length. Returns 0 (covered), 1 (contact) or 2 (H halved 60 times in a row, or too
// many macro steps).
template <int NL, bool COL, int PT>
__device__ __forceinline__ int ce_advance(double (&y)[6], double Ltot, bool check, bool alive,
                                          double fR, const CeLane &L, CeShared &sh,
                                          const CePartner (&pr)[kCeRegPartners], int &buf,
                                          double &done, double &Hc) {
  double t = 0.0, H = Ltot;
  int halvings = 0, macro = 0;
  while (fabs(Ltot - t) > 0.0) {
    if (++macro > kMaxMacroSteps) return 2;
    if (fabs(H) > fabs(Ltot - t)) H = Ltot - t;
    double y1[6];
    const int c = ce_attempt<NL, PT>(y, H, COL ? alive : true, L, sh, pr, buf, y1);
    if (c < 0) {
      H = H / 2.0;
      if (++halvings > 60) return 2;
      continue;
    }
    halvings = 0;
    if (COL && check && ce_contact(y1, fR, L, sh, pr) >= 0) {
      done = t;
      Hc = H;
      return 1;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) y[i] = y1[i];
    if (t + H == t) break;   // the remaining interval is below the resolution of t
    t = t + H;
    if (c <= 2) H = H * 2.5;
    else if (c == 3) H = H * 1.5;
    else H = H * 1.2;
  }
  return 0;
}

// stats (device uint64 [6]): [0] groups integrated, [1] largest group, [2] bodies in groups, [3]
// groups above 64 bodies (drifted on Kepler orbits only), [4] groups whose integration did not
// finish (step halved 60 times in a row, or too many macro steps).
//
// Collisions (col.radius not null): two live members are in contact when their distance is below
// f (R_i + R_j). The integration stops at the first accepted step that ends in contact, the first
// contact time inside that step is found by bisection on the step length (each trial integrating
// from the step's start; at most kMaxBisections halvings, fewer when the interval can no longer be
// split), and the contact pair of lowest member ranks merges there: the lower body index keeps
// the summed mass, the summed volume and the centre-of-mass position and velocity; the other
// becomes massless, of zero radius, parked on a circular orbit of radius kParkRadius about the
// central mass at the angle 2 pi j/n, and is held fixed for the rest of the drift. Each merger is
// logged as {step, survivor, removed} with its time within the drift.
template <int NL, bool COL>
__device__ __forceinline__ void ce_group(
    int w, CeShared &sh, double4 *__restrict__ xm, double4 *__restrict__ v,
    const double4 *__restrict__ thr, const int *__restrict__ gmem, const int *__restrict__ gstart,
    const int *__restrict__ gsize, const int *__restrict__ groot, double G, double m0, double f_in,
    double h, double tol, unsigned long long *__restrict__ stats, const CeCollide &col,
    const LevelThr &lt, int slice) {
  const int r = groot[w];
  const int k = gsize[r];
  const int base = gstart[r];
  const double Gm0 = G * m0;
  if (k > 64) {
    // too large for one wave: Kepler orbits only, and reported (with member slices of fixed length
    // the caller drifts these members itself)
    for (int q = threadIdx.x; q < (slice ? 0 : k); q += 64 * kCeWaves) {
      const int b = gmem[base + q];
      double4 p = xm[b], u = v[b];
      kepler_advance(p.x, p.y, p.z, u.x, u.y, u.z, Gm0, h);
      xm[b] = p;
      v[b] = u;
    }
    if (threadIdx.x == 0) atomicAdd(stats + 3, 1ull);
    return;
  }
  CeLane L;
  L.k = k;
  L.wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int kp = 1;
  while (kp < k) kp <<= 1;
  L.P = min(kp, 64 / kp);
  L.slot = lane / L.P;
  L.rep = lane & (L.P - 1);
  L.iters = (k + L.P - 1) / L.P;
  L.act = L.slot < k;
  L.Gm0 = Gm0;
  L.f_in = f_in;
  L.tol = tol;
  L.nl = lt.nl;
  const int b = gmem[base + (L.act ? L.slot : 0)];
  const double4 p0 = xm[b], u0 = v[b];
  L.rc = thr[b].x;
  L.ispan = 1.0 / ((1.0 - f_in) * L.rc);
  L.rank = 0;
  for (int q = 0; q < k; ++q) L.rank += gmem[base + q] < b;
  const bool collide = COL;
  const double R0 = collide ? col.radius[b] : 0.0;
  if (L.wv == 0 && L.rep == 0 && L.act) {
    sh.owner[L.rank] = L.slot;
    sh.body[L.rank] = b;
    sh.mass[L.rank] = p0.w;
    sh.rad[L.rank] = R0;
    sh.mem[L.rank] = CeMember{G * p0.w, L.rc, L.ispan, col.f * R0};
    for (int l = 0; l < lt.nl; ++l) {
      const double rcl = l == 0 ? L.rc : lt.thr[l][b].x;
      sh.lrc[l][L.rank] = rcl;
      sh.lisp[l][L.rank] = 1.0 / ((1.0 - f_in) * rcl);
    }
  }
  __syncthreads();
  CePartner pr[kCeRegPartners];
#pragma unroll
  for (int u = 0; u < kCeRegPartners; ++u)
    pr[u] = ce_partner(L.rep + u * L.P, L, sh);
  bool alive = true;
  double fR = col.f * R0;
  double y[6] = {p0.x, p0.y, p0.z, u0.x, u0.y, u0.z};
  double y0[6] = {0, 0, 0, 0, 0, 0};
  int status = 0, buf = 0, phase = 0, bis = 0;
  double t = 0.0, lo = 0.0, hi = 0.0, mid = 0.0;
  // phase 0: integrate the rest of the drift (with contact tests when colliding); phase 1: a
  // bisection trial from y0 over mid; phase 2: from y0 to the contact time hi, then merge
  while (true) {
    double L_int = h - t;
    if (phase != 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i) y[i] = y0[i];
      L_int = phase == 1 ? mid : hi;
    }
    double done = 0.0, Hc = 0.0;
    // the replica layout of groups of up to 8 bodies is a compile-time constant of the integrator
    const bool chk = collide && phase == 0;
    int st;
    if (L.iters == 1 && L.P == 2)
      st = ce_advance<NL, COL, 2>(y, L_int, chk, alive, fR, L, sh, pr, buf, done, Hc);
    else if (L.iters == 1 && L.P == 4)
      st = ce_advance<NL, COL, 4>(y, L_int, chk, alive, fR, L, sh, pr, buf, done, Hc);
    else if (L.iters == 1 && L.P == 8)
      st = ce_advance<NL, COL, 8>(y, L_int, chk, alive, fR, L, sh, pr, buf, done, Hc);
    else
      st = ce_advance<NL, COL, 0>(y, L_int, chk, alive, fR, L, sh, pr, buf, done, Hc);
    if (st == 2) { status = 1; break; }
    if (phase == 0) {
      if (st == 0) break;
      t = t + done;
#pragma unroll
      for (int i = 0; i < 6; ++i) y0[i] = y[i];
      lo = 0.0;
      hi = Hc;
      bis = 0;
    } else if (phase == 1) {
      if (ce_contact(y, fR, L, sh, pr) >= 0) hi = mid; else lo = mid;
      ++bis;
    } else {
      t = t + hi;
      const int key = ce_contact(y, fR, L, sh, pr);
      if (key >= 0) {
        const int ra = key >> 6, rb = key & 63;
        const int sa = sh.owner[ra] * L.P, sb = sh.owner[rb] * L.P;
        const double ma = sh.mass[ra], mb = sh.mass[rb];
        const double M = ma + mb;
        double ya[6], yb[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          ya[i] = __shfl(y[i], sa, 64);
          yb[i] = __shfl(y[i], sb, 64);
        }
        const double Ra = sh.rad[ra], Rb = sh.rad[rb];
        const double Rm = cbrt(Ra * Ra * Ra + Rb * Rb * Rb);
        const int ba = sh.body[ra], bb = sh.body[rb];
        if (L.rank == ra && L.act) {
#pragma unroll
          for (int i = 0; i < 6; ++i) y[i] = (ma * ya[i] + mb * yb[i]) / M;
          fR = col.f * Rm;
        }
        if (L.rank == rb && L.act) {
          const double th = 2.0 * M_PI * (double)bb / (double)col.n;
          const double vc = sqrt(Gm0 / kParkRadius);
          y[0] = kParkRadius * cos(th);
          y[1] = kParkRadius * sin(th);
          y[2] = 0.0;
          y[3] = -vc * sin(th);
          y[4] = vc * cos(th);
          y[5] = 0.0;
          alive = false;
          fR = 0.0;
        }
        __syncthreads();   // every wave is past its last read of the member values
        if (threadIdx.x == 0) {
          sh.mass[ra] = M;
          sh.mass[rb] = 0.0;
          sh.rad[ra] = Rm;
          sh.rad[rb] = 0.0;
          sh.mem[ra].Gm = G * M;
          sh.mem[ra].fR = col.f * Rm;
          sh.mem[rb].Gm = 0.0;
          sh.mem[rb].fR = 0.0;
          const unsigned long long e = atomicAdd(col.count, 1ull);
          if (e < (unsigned long long)col.cap) {
            col.merges[3 * e] = col.step;
            col.merges[3 * e + 1] = ba;
            col.merges[3 * e + 2] = bb;
            col.mtime[e] = t;
          }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kCeRegPartners; ++u)
          pr[u] = ce_partner(L.rep + u * L.P, L, sh);
      }
      phase = 0;
      if (!(fabs(h - t) > 0.0)) break;
      continue;
    }
    // next bisection trial, or the final advance to the contact time
    mid = 0.5 * (lo + hi);
    phase = (bis < kMaxBisections && mid > lo && mid < hi) ? 1 : 2;
  }
  if (L.wv == 0 && L.rep == 0 && L.act) {
    xm[b] = make_double4(y[0], y[1], y[2], sh.mass[L.rank]);
    v[b] = make_double4(y[3], y[4], y[5], u0.w);
    if (collide) col.radius[b] = sh.rad[L.rank];
  }
  if (threadIdx.x == 0) {
    atomicAdd(stats + 0, 1ull);
    atomicMax(stats + 1, (unsigned long long)k);
    atomicAdd(stats + 2, (unsigned long long)k);
    if (status) atomicAdd(stats + 4, 1ull);
  }
}

// Resident workgroups take groups from a queue (counter[2]) until all counter[0] groups are done.
template <int NL, bool COL>
__global__ __launch_bounds__(64 * kCeWaves) void k_ce_drift(
    double4 *__restrict__ xm, double4 *__restrict__ v, const double4 *__restrict__ thr,
    const int *__restrict__ gmem, const int *__restrict__ gstart, const int *__restrict__ gsize,
    const int *__restrict__ groot, int *__restrict__ counter, double G, double m0, double f_in,
    double h, double tol, unsigned long long *__restrict__ stats, CeCollide col, LevelThr lt,
    int slice) {
  __shared__ CeShared sh;
  __shared__ int next;
  const int ng = counter[0];
  while (true) {
    if (threadIdx.x == 0) next = atomicAdd(counter + 2, 1);
    __syncthreads();
    const int w = next;
    __syncthreads();
    if (w >= ng) break;
    ce_group<NL, COL>(w, sh, xm, v, thr, gmem, gstart, gsize, groot, G, m0, f_in, h, tol, stats, col, lt,
                      slice);
    __syncthreads();
  }
}

hipError_t launch_group_lists(const int *label, int n, int *in, int *gsize, int *gstart, int *gfill,
                              int *gmem, int *groot, int *counter, bool counted, hipStream_t st,
                              const int *deg, int *skip) {
  if (!counted) {
    hipLaunchKernelGGL(k_gzero, dim3(nblocks(n > kGroupCounters ? n : kGroupCounters)), dim3(kBlock),
                       0, st, n, gsize, gfill, counter);
    hipLaunchKernelGGL(k_gcount, dim3(nblocks(n)), dim3(kBlock), 0, st, label, n, gsize);
  }
  hipLaunchKernelGGL(k_galloc, dim3(nblocks(n)), dim3(kBlock), 0, st, label, gsize, n, in, gstart,
                     groot, counter, deg, skip);
  hipLaunchKernelGGL(k_gfill, dim3(nblocks(n)), dim3(kBlock), 0, st, label, in, n, gstart, gfill,
                     gmem);
  return hipGetLastError();
}

hipError_t launch_ce_drift(double4 *xm, double4 *v, const double4 *thr, const int *gmem,
                           const int *gstart, const int *gsize, const int *groot, int *counter,
                           int max_groups, double G, double m0, double f_in, double h, double tol,
                           unsigned long long *stats, const CeCollide &col, const LevelThr &lt,
                           hipStream_t st, int slice) {
  // resident workgroups only: the queue hands out the groups (the device count is not known here)
  if (max_groups <= 0) return hipSuccess;
  const bool col_on = col.radius != nullptr;
#define NBK_CE(A, B)                                                                                \
  do {                                                                                              \
    static int resident = 0;                                                                        \
    if (resident == 0) {                                                                            \
      int dev = 0, per = 0;                                                                         \
      hipDeviceProp_t prop;                                                                         \
      hipError_t e = hipGetDevice(&dev);                                                            \
      if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);                                  \
      if (e == hipSuccess)                                                                          \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_ce_drift<A, B>, 64 * kCeWaves, 0); \
      if (e != hipSuccess) return e;                                                                \
      resident = std::max(1, per) * prop.multiProcessorCount;                                       \
    }                                                                                               \
    hipLaunchKernelGGL((k_ce_drift<A, B>), dim3(std::min(max_groups, resident)), dim3(64 * kCeWaves), \
                       0, st, xm, v, thr, gmem, gstart, gsize, groot, counter, G, m0, f_in, h, tol,  \
                       stats, col, lt, slice);                                                      \
  } while (0)
  if (lt.nl == 1) { if (col_on) NBK_CE(1, true); else NBK_CE(1, false); }
  else if (lt.nl == 2) { if (col_on) NBK_CE(2, true); else NBK_CE(2, false); }
  else { if (col_on) NBK_CE(0, true); else NBK_CE(0, false); }
#undef NBK_CE
  return hipGetLastError();
}

}  // namespace nbk
