// Plain CPU oracle of the hybrid-symplectic planetesimal step (democratic heliocentric
// coordinates, H = H_A + H_B + H_C; Grimm & Stadel, "Terrestrial planet formation in the era
// of GPU computing", section "The hybrid symplectic integrator", equations Ha, Hb, Hc, rcrit).
//
// TEST INFRASTRUCTURE ONLY. This file is the slow, obviously-correct reference that the HIP
// library is checked against. Only the test suite, the smoke check and the benchmark's CPU
// baseline may load it; the library never does. It shares no code, header or constant with
// the HIP path.
//
// Arithmetic: binary64 with round-to-nearest, no fast-math, no contraction (-ffp-contract=off);
// fma only where written. Every routine is a template over the scalar type so that the same
// definition also runs in long double, __float128 (accuracy pins) and forward-mode dual numbers
// (gradient reference). Sums over bodies run in ascending index order with Neumaier's
// compensated summation (Neumaier 1974) for binary64, plain summation otherwise.
//
// Readings of points the paper leaves open (each is listed in the design notes):
//  * K(r): the changeover of Chambers (1999), the paper cited for the rcrit equation:
//    y = (r - f_in rc)/((1 - f_in) rc) clamped to [0,1], K = y^2/(2y^2 - 2y + 1), f_in = 0.1.
//  * The kick is the gradient of H_B with rc held fixed: w = K/r^3 - K'(r)/r^2.
//  * rc_i = max(n1 R_Hill,i, n2 dt |v_i|), R_Hill,i = |x_i| (m_i/(3 m0))^(1/3); pair radius
//    rc_ij = max(rc_i, rc_j); rc is computed once from the state at the start of a call and held.
//  * Encounter predicate, exactly in binary64: with d = x_j - x_i and
//    r2 = fma(dz,dz,fma(dy,dy,dx*dx)), the pair is close iff
//    (r2*r2)*r2 < max(H_i,H_j) or r2 < max(V_i,V_j), where
//    H_i = cH*((r2_i*r2_i)*r2_i)*(mu_i*mu_i), cH = ((n1*n1*n1)*(n1*n1*n1))/9, mu_i = m_i/m0,
//    V_i = cV*vv_i, cV = (n2*dt)*(n2*dt), vv_i = fma(vz,vz,fma(vy,vy,vx*vx)).
//    In real arithmetic this is r_ij < max(rc_i, rc_j).
//  * Step: B(dt/2) C(dt/2) A(dt) C(dt/2) B(dt/2) (operator order of the democratic heliocentric
//    method the paper cites); A is the Kepler drift about mu = G m0. The plain step leaves the
//    [1-K] part of H_A out; the hybrid steps integrate it for every close-encounter group
//    (Gragg-Bulirsch-Stoer in long double), optionally through intermediate changeover levels and
//    with collisions as perfect mergers (readings at those routines below).
//  * Kepler drift: f and g functions with the eccentric-anomaly difference form of Kepler's
//    equation (elliptic) or its hyperbolic analogue, solved by safeguarded Newton iteration in
//    long double.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdio>
#include <vector>
#include <algorithm>
#include <quadmath.h>
#include <omp.h>

namespace orc {

// ---------------------------------------------------------------- scalar types and math
template <class B> struct Dual {
  B v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(B a, B b) : v(a), d(b) {}
};
template <class B> Dual<B> operator+(Dual<B> a, Dual<B> b) { return {a.v + b.v, a.d + b.d}; }
template <class B> Dual<B> operator-(Dual<B> a, Dual<B> b) { return {a.v - b.v, a.d - b.d}; }
template <class B> Dual<B> operator-(Dual<B> a) { return {-a.v, -a.d}; }
template <class B> Dual<B> operator*(Dual<B> a, Dual<B> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class B> Dual<B> operator/(Dual<B> a, Dual<B> b) {
  B q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <class B> Dual<B> &operator+=(Dual<B> &a, Dual<B> b) { a = a + b; return a; }
template <class B> Dual<B> &operator-=(Dual<B> &a, Dual<B> b) { a = a - b; return a; }
template <class B> Dual<B> &operator*=(Dual<B> &a, Dual<B> b) { a = a * b; return a; }
template <class B> Dual<B> operator+(Dual<B> a, double b) { return a + Dual<B>(b); }
template <class B> Dual<B> operator-(Dual<B> a, double b) { return a - Dual<B>(b); }
template <class B> Dual<B> operator*(Dual<B> a, double b) { return a * Dual<B>(b); }
template <class B> Dual<B> operator/(Dual<B> a, double b) { return a / Dual<B>(b); }
template <class B> Dual<B> operator+(double a, Dual<B> b) { return Dual<B>(a) + b; }
template <class B> Dual<B> operator-(double a, Dual<B> b) { return Dual<B>(a) - b; }
template <class B> Dual<B> operator*(double a, Dual<B> b) { return Dual<B>(a) * b; }
template <class B> Dual<B> operator/(double a, Dual<B> b) { return Dual<B>(a) / b; }

typedef Dual<double> dual;
typedef __float128 quad;

inline double val(double a) { return a; }
inline double val(long double a) { return (double)a; }
inline double val(quad a) { return (double)a; }
template <class B> inline double val(Dual<B> a) { return (double)a.v; }

inline double msqrt(double a) { return std::sqrt(a); }
inline long double msqrt(long double a) { return sqrtl(a); }
inline quad msqrt(quad a) { return sqrtq(a); }
inline double mcbrt(double a) { return std::cbrt(a); }
inline long double mcbrt(long double a) { return cbrtl(a); }
inline quad mcbrt(quad a) { return cbrtq(a); }
inline double msin(double a) { return std::sin(a); }
inline long double msin(long double a) { return sinl(a); }
inline quad msin(quad a) { return sinq(a); }
inline double mcos(double a) { return std::cos(a); }
inline long double mcos(long double a) { return cosl(a); }
inline quad mcos(quad a) { return cosq(a); }
inline double msinh(double a) { return std::sinh(a); }
inline long double msinh(long double a) { return sinhl(a); }
inline quad msinh(quad a) { return sinhq(a); }
inline double mcosh(double a) { return std::cosh(a); }
inline long double mcosh(long double a) { return coshl(a); }
inline quad mcosh(quad a) { return coshq(a); }
template <class B> Dual<B> msqrt(Dual<B> a) { B s = msqrt(a.v); return {s, a.d / (B(2) * s)}; }
template <class B> Dual<B> mcbrt(Dual<B> a) { B c = mcbrt(a.v); return {c, a.d / (B(3) * c * c)}; }
template <class B> Dual<B> msin(Dual<B> a) { return {msin(a.v), a.d * mcos(a.v)}; }
template <class B> Dual<B> mcos(Dual<B> a) { return {mcos(a.v), -a.d * msin(a.v)}; }
template <class B> Dual<B> msinh(Dual<B> a) { return {msinh(a.v), a.d * mcosh(a.v)}; }
template <class B> Dual<B> mcosh(Dual<B> a) { return {mcosh(a.v), a.d * msinh(a.v)}; }
// fma: exact single rounding where the type has one; for duals the product rule.
inline double mfma(double a, double b, double c) { return std::fma(a, b, c); }
inline long double mfma(long double a, long double b, long double c) { return fmal(a, b, c); }
inline quad mfma(quad a, quad b, quad c) { return fmaq(a, b, c); }
template <class B> Dual<B> mfma(Dual<B> a, Dual<B> b, Dual<B> c) { return a * b + c; }

template <class T> inline T mabs(T a) { return val(a) < 0 ? T(0) - a : a; }
template <class T> inline T mmax(T a, T b) { return val(a) >= val(b) ? a : b; }
template <class T> inline T mmin(T a, T b) { return val(a) <= val(b) ? a : b; }
template <class T> inline double teps() { return 2.220446049250313e-16; }
template <> inline double teps<long double>() { return 1.0842021724855044e-19; }
template <> inline double teps<quad>() { return 1.925929944387236e-34; }

// Compensated sum (Neumaier 1974) for binary64; plain sum for any other type.
template <class T> struct Acc {
  T s = T(0);
  void add(T x) { s = s + x; }
  T get() const { return s; }
};
template <> struct Acc<double> {
  double s = 0, c = 0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
  }
  double get() const { return s + c; }
};

// ---------------------------------------------------------------- parameters
// nl: number of changeover levels whose [1 - K_l] factors weight the close-encounter pair term
// (1 without intermediate levels).
struct Params { double G, m0, dt, n1, n2, f_in; int nl = 1; };

// ---------------------------------------------------------------- critical radius (eq. rcrit)
// Per body: rc_i (used by the changeover), and the exact-predicate thresholds H_i, V_i.
// Always binary64: the thresholds are fixed parameters of the kick, not differentiated.
static void thresholds(int64_t n, const double *x, const double *v, const double *m,
                       const Params &p, double *rc, double *H, double *V) {
  const double cH = ((p.n1 * p.n1 * p.n1) * (p.n1 * p.n1 * p.n1)) / 9.0;
  const double t = p.n2 * p.dt;
  const double cV = t * t;
  for (int64_t i = 0; i < n; i++) {
    const double *xi = x + 3 * i, *vi = v + 3 * i;
    double r2 = std::fma(xi[2], xi[2], std::fma(xi[1], xi[1], xi[0] * xi[0]));
    double mu = m[i] / p.m0;
    double vv = std::fma(vi[2], vi[2], std::fma(vi[1], vi[1], vi[0] * vi[0]));
    H[i] = (cH * ((r2 * r2) * r2)) * (mu * mu);
    V[i] = cV * vv;
    double rhill = std::sqrt(r2) * std::cbrt(mu / 3.0);
    rc[i] = std::max(p.n1 * rhill, t * std::sqrt(vv));
  }
}

// Exact binary64 encounter predicate on the positions' binary64 values.
static inline bool close_pair(const double *xi, const double *xj, double Hi, double Hj,
                              double Vi, double Vj, double *r2out) {
  double dx = xj[0] - xi[0], dy = xj[1] - xi[1], dz = xj[2] - xi[2];
  double r2 = std::fma(dz, dz, std::fma(dy, dy, dx * dx));
  *r2out = r2;
  return ((r2 * r2) * r2 < std::max(Hi, Hj)) || (r2 < std::max(Vi, Vj));
}

// ---------------------------------------------------------------- changeover K(y)
template <class T> static void changeover(T y, T *K, T *dKdy) {
  if (val(y) <= 0) { *K = T(0); *dKdy = T(0); return; }
  if (val(y) >= 1) { *K = T(1); *dKdy = T(0); return; }
  T D = T(2) * y * y - T(2) * y + T(1);
  *K = y * y / D;
  *dKdy = T(2) * y * (T(1) - y) / (D * D);
}

// Pair weight w(r) such that the H_B acceleration of i due to j is G m_j w d, d = x_j - x_i.
template <class T> static T pair_weight(T r2, bool close, double rcij, double f_in) {
  T r = msqrt(r2);
  T r3 = r2 * r;
  if (!close) return T(1) / r3;
  T y = (r - T(f_in * rcij)) / T((1.0 - f_in) * rcij);
  T K, dKdy;
  changeover(y, &K, &dKdy);
  T dKdr = dKdy / T((1.0 - f_in) * rcij);
  return K / r3 - dKdr / r2;
}

// ---------------------------------------------------------------- H_B kick (eq. Hb)
// acc[i] = G sum_{j != i} m_j w_ij (x_j - x_i); acc_ce = the complementary [1-K] part, so that
// acc + acc_ce is the plain Newtonian pull of the other planetesimals; l1[i] =
// G sum_j m_j |w_ij| r_ij, the scale used for relative-error statements.
template <class T>
static void kick_acc(int64_t n, const T *x, const T *m, const double *rc, const double *H,
                     const double *V, const Params &p, T *acc, T *acc_ce, double *l1) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; i++) {
    double xi_d[3] = {val(x[3 * i]), val(x[3 * i + 1]), val(x[3 * i + 2])};
    Acc<T> a[3], ace[3];
    double l1s = 0;
    for (int64_t j = 0; j < n; j++) {
      if (j == i) continue;
      double xj_d[3] = {val(x[3 * j]), val(x[3 * j + 1]), val(x[3 * j + 2])};
      double r2d;
      bool close = close_pair(xi_d, xj_d, H[i], H[j], V[i], V[j], &r2d);
      T d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
      T r2 = mfma(d[2], d[2], mfma(d[1], d[1], d[0] * d[0]));
      T w = pair_weight(r2, close, std::max(rc[i], rc[j]), p.f_in);
      T s = T(p.G) * m[j] * w;
      for (int k = 0; k < 3; k++) a[k].add(s * d[k]);
      if (close) {
        T sn = T(p.G) * m[j] / (r2 * msqrt(r2));
        for (int k = 0; k < 3; k++) ace[k].add((sn - s) * d[k]);
      }
      l1s += p.G * val(m[j]) * std::fabs(val(w)) * std::sqrt(val(r2));
    }
    for (int k = 0; k < 3; k++) {
      acc[3 * i + k] = a[k].get();
      if (acc_ce) acc_ce[3 * i + k] = ace[k].get();
    }
    if (l1) l1[i] = l1s;
  }
}

// ---------------------------------------------------------------- encounter list
// All close pairs (i < j), in ascending (i, j) order. Returns the true count; writes at most cap.
static int64_t encounters(int64_t n, const double *x, const double *H, const double *V,
                          int64_t cap, int32_t *pairs) {
  std::vector<std::vector<int32_t>> rows(n);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; i++)
    for (int64_t j = i + 1; j < n; j++) {
      double r2;
      if (close_pair(x + 3 * i, x + 3 * j, H[i], H[j], V[i], V[j], &r2)) rows[i].push_back((int32_t)j);
    }
  int64_t c = 0;
  for (int64_t i = 0; i < n; i++)
    for (int32_t j : rows[i]) {
      if (c < cap) { pairs[2 * c] = (int32_t)i; pairs[2 * c + 1] = j; }
      c++;
    }
  return c;
}

// ---------------------------------------------------------------- H_C jump (eq. Hc)
template <class T> static void jump(int64_t n, T *x, const T *v, const T *m, const Params &p, T h) {
  Acc<T> P[3];
  for (int64_t j = 0; j < n; j++)
    for (int k = 0; k < 3; k++) P[k].add(m[j] * v[3 * j + k]);
  T s[3];
  for (int k = 0; k < 3; k++) s[k] = h * (P[k].get() / T(p.m0));
  for (int64_t i = 0; i < n; i++)
    for (int k = 0; k < 3; k++) x[3 * i + k] = x[3 * i + k] + s[k];
}

// ---------------------------------------------------------------- H_A Kepler drift (eq. Ha)
// Advances (x, v) of one body along its two-body orbit about mu for time dt with the f and g
// functions. Returns 0, or 1 if the anomaly iteration did not converge, 2 for an orbit so close
// to parabolic that neither branch applies.
template <class T> static int kepler(T *x, T *v, double mu_d, double dt_d) {
  T mu = T(mu_d), dt = T(dt_d);
  T r0 = msqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  T v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  T u = x[0] * v[0] + x[1] * v[1] + x[2] * v[2];
  T alpha = T(2) / r0 - v2 / mu;  // 1/a
  double ar = val(alpha) * val(r0);
  if (std::fabs(ar) < 1e-10) return 2;
  const double tol = 8 * teps<T>();
  T f, g, fd, gd;
  int status = 0;
  if (val(alpha) > 0) {
    T a = T(1) / alpha;
    T n = msqrt(mu * alpha * alpha * alpha);
    T c = T(1) - r0 * alpha;        // e cos E0
    T s = u / msqrt(mu * a);        // e sin E0
    T M = n * dt;
    auto F = [&](T E) { return E - c * msin(E) + s * (T(1) - mcos(E)) - M; };
    auto Fp = [&](T E) { return T(1) - c * mcos(E) + s * msin(E); };
    // root bracket: |c sin E - s (1 - cos E)| <= |c| + 2|s| < 3 for e < 1
    T lo = M - T(3), hi = M + T(3), E = M;
    int it = 0;
    for (; it < 200; it++) {
      T Fx = F(E);
      if (val(Fx) > 0) hi = E; else lo = E;
      T En = E - Fx / Fp(E);
      if (!(val(En) > val(lo) && val(En) < val(hi))) En = (lo + hi) * 0.5;
      double step = std::fabs(val(En - E));
      E = En;
      if (step <= tol * (1 + std::fabs(val(E)))) break;
    }
    if (it == 200) status = 1;
    for (int k = 0; k < 2; k++) E = E - F(E) / Fp(E);  // carries exact implicit derivatives
    T sE = msin(E), cE = mcos(E);
    T hs = msin(E * 0.5);
    T omc = T(2) * hs * hs;  // 1 - cos E
    T r = a * (T(1) - c * cE + s * sE);
    f = T(1) - (a / r0) * omc;
    g = dt - (E - sE) / n;
    fd = T(0) - msqrt(mu * a) * sE / (r * r0);
    gd = T(1) - (a / r) * omc;
  } else {
    T A = T(0) - T(1) / alpha;  // |a|
    T n = msqrt(mu / (A * A * A));
    T c = T(1) + r0 / A;            // e cosh H0
    T s = u / msqrt(mu * A);        // e sinh H0
    T M = n * dt;
    auto F = [&](T H) { return c * msinh(H) + s * (mcosh(H) - T(1)) - H - M; };
    auto Fp = [&](T H) { return c * mcosh(H) + s * msinh(H) - T(1); };
    T lo = T(0), hi = T(0);
    if (val(M) >= 0) { hi = T(1); while (val(F(hi)) < 0) hi = hi * 2.0; }
    else { lo = T(-1); while (val(F(lo)) > 0) lo = lo * 2.0; }
    T H = (lo + hi) * 0.5;
    int it = 0;
    for (; it < 400; it++) {
      T Fx = F(H);
      if (val(Fx) > 0) hi = H; else lo = H;
      T Hn = H - Fx / Fp(H);
      if (!(val(Hn) > val(lo) && val(Hn) < val(hi))) Hn = (lo + hi) * 0.5;
      double step = std::fabs(val(Hn - H));
      H = Hn;
      if (step <= tol * (1 + std::fabs(val(H)))) break;
    }
    if (it == 400) status = 1;
    for (int k = 0; k < 2; k++) H = H - F(H) / Fp(H);
    T sH = msinh(H), cH = mcosh(H);
    T r = A * (c * cH + s * sH - T(1));
    f = T(1) - (A / r0) * (cH - T(1));
    g = dt - (sH - H) / n;
    fd = T(0) - msqrt(mu * A) * sH / (r * r0);
    gd = T(1) - (A / r) * (cH - T(1));
  }
  T xn[3], vn[3];
  for (int k = 0; k < 3; k++) {
    xn[k] = f * x[k] + g * v[k];
    vn[k] = fd * x[k] + gd * v[k];
  }
  for (int k = 0; k < 3; k++) { x[k] = xn[k]; v[k] = vn[k]; }
  return status;
}

// Drift of all bodies. binary64 states are advanced in long double and rounded once.
template <class T> static int drift_all(int64_t n, T *x, T *v, const Params &p, double h, uint32_t *st) {
  int worst = 0;
  for (int64_t i = 0; i < n; i++) {
    int s = kepler<T>(x + 3 * i, v + 3 * i, p.G * p.m0, h);
    if (st) st[i] = (uint32_t)s;
    worst = std::max(worst, s);
  }
  return worst;
}
template <> int drift_all<double>(int64_t n, double *x, double *v, const Params &p, double h, uint32_t *st) {
  int worst = 0;
  for (int64_t i = 0; i < n; i++) {
    long double xl[3], vl[3];
    for (int k = 0; k < 3; k++) { xl[k] = x[3 * i + k]; vl[k] = v[3 * i + k]; }
    int s = kepler<long double>(xl, vl, p.G * p.m0, h);
    for (int k = 0; k < 3; k++) { x[3 * i + k] = (double)xl[k]; v[3 * i + k] = (double)vl[k]; }
    if (st) st[i] = (uint32_t)s;
    worst = std::max(worst, s);
  }
  return worst;
}

// ---------------------------------------------------------------- one call of nsteps steps
// B(h) C(h) A(dt) C(h) B(h) per step, h = dt/2, thresholds from the state at call start.
// Close-encounter groups: the connected components of the graph whose edges are the close pairs
// (the bodies that the hybrid method hands to its close-encounter integrator together). Every body
// is labelled with the smallest index in its component: bodies are visited in ascending order and
// a breadth-first search from each body not yet reached labels its whole component with it.
// Returns the number of components with at least two bodies; pairs with an index outside 0..n-1
// or with i == j are not edges and are counted in *ignored.
static int64_t groups_bfs(int64_t n, const int32_t *pairs, int64_t npairs, int32_t *label, int64_t *ignored) {
  std::vector<std::vector<int64_t>> adj((size_t)n);
  int64_t bad = 0;
  for (int64_t k = 0; k < npairs; k++) {
    const int64_t i = pairs[2 * k], j = pairs[2 * k + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) {
      bad++;
      continue;
    }
    adj[(size_t)i].push_back(j);
    adj[(size_t)j].push_back(i);
  }
  for (int64_t i = 0; i < n; i++) label[i] = -1;
  int64_t groups = 0;
  std::vector<int64_t> queue;
  for (int64_t s = 0; s < n; s++) {
    if (label[s] >= 0) continue;
    label[s] = (int32_t)s;
    queue.assign(1, s);
    for (size_t q = 0; q < queue.size(); q++)
      for (int64_t t : adj[(size_t)queue[q]])
        if (label[t] < 0) {
          label[t] = (int32_t)s;
          queue.push_back(t);
        }
    if (queue.size() >= 2) groups++;
  }
  if (ignored) *ignored = bad;
  return groups;
}

// ---------------------------------------------------------------- close-encounter drift (eq. Ha)
// H_A in full: sum_i (p_i^2/2m_i - G m0 m_i/r_i) - sum_{i<j} G m_i m_j [1 - K(r_ij)]/r_ij. The
// bodies of a close-encounter group move under the equations of motion of H_A restricted to the
// group:
//   dx_i/dt = v_i,
//   dv_i/dt = -G m0 x_i/|x_i|^3 + G sum_{j in group, j != i} m_j ((1 - K)/r^3 + K'(r)/r^2) d_ij,
// with d_ij = x_j - x_i: the pair term is minus the gradient of the [1 - K] part of the pair
// potential, the complement of the kick's weight, and vanishes for r >= rc_ij. Bodies in no group
// keep the Kepler drift.
// Product of the changeover complements of the levels 0..nl-1 for a pair at distance q,
// W = prod_l (1 - K_l(q)), and dW/dq; rcs[l] = rc_l,ij of level l.
template <class T>
static void level_weight(T q, const double *rcs, int nl, const Params &p, T *W, T *dW) {
  T w = T(1), dw = T(0);
  for (int l = 0; l < nl; l++) {
    const T span = T((1.0 - p.f_in) * rcs[l]);
    T K, dKdy;
    changeover((q - T(p.f_in * rcs[l])) / span, &K, &dKdy);
    const T dK = dKdy / span;
    dw = dw * (T(1) - K) - w * dK;
    w = w * (T(1) - K);
  }
  *W = w;
  *dW = dw;
}

// The equations of motion of a group under H_A: Kepler about the central mass plus the pair term
// of the potential -G m_i m_j W(r)/r, W = prod over the levels of [1 - K_l] (one level without
// intermediate levels: the [1 - K] part). rc holds the members' critical radii level by level
// ([nl][k]).
template <class T>
static void ce_rhs(int k, const T *y, const double *m, const double *rc, const bool *alive, const Params &p,
                   T *f) {
  const T *x = y, *v = y + 3 * k;
  double rcs[8];
  for (int i = 0; i < k; i++) {
    if (!alive[i]) {           // a body merged away is held fixed
      for (int l = 0; l < 3; l++) f[3 * i + l] = f[3 * k + 3 * i + l] = T(0);
      continue;
    }
    T r2 = x[3 * i] * x[3 * i] + x[3 * i + 1] * x[3 * i + 1] + x[3 * i + 2] * x[3 * i + 2];
    T r = msqrt(r2);
    T s = T(0) - T(p.G * p.m0) / (r2 * r);
    T a[3] = {s * x[3 * i], s * x[3 * i + 1], s * x[3 * i + 2]};
    for (int j = 0; j < k; j++) {
      if (j == i) continue;
      T d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
      T q2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      T q = msqrt(q2);
      if (val(q) >= std::max(rc[i], rc[j])) continue;     // beyond rc_0: W = 0
      for (int l = 0; l < p.nl; l++) rcs[l] = std::max(rc[l * k + i], rc[l * k + j]);
      T W, dW;
      level_weight(q, rcs, p.nl, p, &W, &dW);
      // minus the gradient of -G m_i m_j W/r with respect to x_i, divided by m_i
      T c = T(p.G * m[j]) * (W / (q2 * q) - dW / q2);
      for (int l = 0; l < 3; l++) a[l] = a[l] + c * d[l];
    }
    for (int l = 0; l < 3; l++) {
      f[3 * i + l] = v[3 * i + l];
      f[3 * k + 3 * i + l] = a[l];
    }
  }
}

// Collisions as perfect mergers (the paper's outcomes of collisions, with the radius factor f of
// its section on the acceleration factor). Two bodies of a group are in contact when their
// distance is below f (R_i + R_j); the merger keeps the lower body index with the summed mass, the
// summed volume (R^3 = R_i^3 + R_j^3) and the centre-of-mass position and velocity, and parks the
// other as a massless body of zero radius on a circular orbit of radius 1e6 about the central mass
// at the angle 2 pi j/n, far from everything.
struct MergeCtx {
  double f;                  // radius factor
  int64_t n;                 // bodies in the system (parking angle)
  int step;                  // step index written to the log
  std::vector<int64_t> *log; // {step, survivor, removed} per merger
  std::vector<long double> *time;   // time within the drift of each merger
};

constexpr double kParkRadius = 1e6;
constexpr int kMaxBisections = 80;   // contact-time bisection: at most 80 halvings of the step

template <class T>
static int contact_pair(int k, const T *y, const double *R, const bool *alive, double f) {
  for (int a = 0; a < k; a++)
    for (int b = a + 1; b < k; b++) {
      if (!alive[a] || !alive[b]) continue;
      T d2 = T(0);
      for (int l = 0; l < 3; l++) {
        const T d = y[3 * b + l] - y[3 * a + l];
        d2 = d2 + d * d;
      }
      const T lim = T(f * (R[a] + R[b]));
      if (val(d2) < val(lim * lim)) return a * k + b;
    }
  return -1;
}

// One Gragg-Bulirsch-Stoer attempt over H from y: modified-midpoint sweeps with n = 2, 4, ..., 16
// substeps, extrapolated to zero substep length as a polynomial in (H/n)^2 (Aitken-Neville). The
// attempt is accepted at the first column c >= 2 whose last two extrapolants agree to tol (relative
// to the group's largest position and velocity of the bodies still present); y1 receives that
// extrapolant. Returns the column, or -1.
template <class T>
static int gbs_attempt(int k, const T *y, const double *m, const double *rc, const bool *alive,
                       const Params &p, T H, double tol, T *y1) {
  const int seq[8] = {2, 4, 6, 8, 10, 12, 14, 16};
  const int D = 6 * k;
  std::vector<T> R(8 * (size_t)D), zm(D), zc(D), zn(D), f(D), est(D);
  T sx = T(0), sv = T(0);
  for (int a = 0; a < k; a++)
    for (int l = 0; l < 3; l++)
      if (alive[a]) {
        sx = mmax(sx, mabs(y[3 * a + l]));
        sv = mmax(sv, mabs(y[3 * k + 3 * a + l]));
      }
  for (int c = 0; c < 8; c++) {
    const int ns = seq[c];
    const T hs = H / T(ns);
    // modified midpoint: z1 = z0 + hs f(z0); z_{s+1} = z_{s-1} + 2 hs f(z_s); end value
    // (z_n + z_{n-1} + hs f(z_n)) / 2
    for (int i = 0; i < D; i++) zm[i] = y[i];
    ce_rhs<T>(k, zm.data(), m, rc, alive, p, f.data());
    for (int i = 0; i < D; i++) zc[i] = zm[i] + hs * f[i];
    for (int s = 1; s < ns; s++) {
      ce_rhs<T>(k, zc.data(), m, rc, alive, p, f.data());
      for (int i = 0; i < D; i++) {
        zn[i] = zm[i] + T(2) * hs * f[i];
        zm[i] = zc[i];
        zc[i] = zn[i];
      }
    }
    ce_rhs<T>(k, zc.data(), m, rc, alive, p, f.data());
    for (int i = 0; i < D; i++) est[i] = (zc[i] + zm[i] + hs * f[i]) / T(2);
    // Aitken-Neville in (H/n)^2: row c from row c - 1
    for (int i = 0; i < D; i++) {
      T cur = est[i];
      for (int j = 1; j <= c; j++) {
        const T old = R[(size_t)(j - 1) * D + i];
        R[(size_t)(j - 1) * D + i] = cur;
        const T ratio = T(seq[c]) / T(seq[c - j]);
        cur = cur + (cur - old) / (ratio * ratio - T(1));
      }
      R[(size_t)c * D + i] = cur;
    }
    if (c >= 2) {
      double err = 0;
      for (int i = 0; i < D; i++) {
        const int body = (i % (3 * k)) / 3;
        if (!alive[body]) continue;
        const T sc = i < 3 * k ? sx : sv;
        err = std::max(err, val(mabs(R[(size_t)c * D + i] - R[(size_t)(c - 1) * D + i]) / sc));
      }
      if (err <= tol) {
        for (int i = 0; i < D; i++) y1[i] = R[(size_t)c * D + i];
        return c;
      }
    }
  }
  return -1;
}

// Integration of y over time L: macro steps from H = L, halved when rejected and doubled after
// acceptance at column c <= 4. With radii given, every accepted step is followed by a contact test,
// and the integration stops at the first step that ends in contact: y then still holds the state at
// that step's start, *done the time covered before it and *Hc its length. Returns 0 (L covered),
// 1 (contact) or 2 (H halved more than 60 times in a row).
template <class T>
static int gbs_advance(int k, T *y, const double *m, const double *rc, const bool *alive, const double *R,
                       const Params &p, T L, double tol, double f, T *done, T *Hc) {
  const int D = 6 * k;
  std::vector<T> y1(D);
  T t = T(0), H = L;
  int halvings = 0;
  while (val(mabs(L - t)) > 0) {
    if (val(mabs(H)) > val(mabs(L - t))) H = L - t;
    const int c = gbs_attempt<T>(k, y, m, rc, alive, p, H, tol, y1.data());
    if (c < 0) {
      H = H / T(2);
      if (++halvings > 60) return 2;
      continue;
    }
    halvings = 0;
    if (R && contact_pair<T>(k, y1.data(), R, alive, f) >= 0) {
      *done = t;
      *Hc = H;
      return 1;
    }
    for (int i = 0; i < D; i++) y[i] = y1[i];
    if (t + H == t) break;            // the remaining interval is below the resolution of t
    t = t + H;
    if (c <= 4) H = H * T(2);
  }
  return 0;
}

// Close-encounter drift of one group over time h (y = [x (3k), v (3k)] in and out). Without
// collisions (mc null) one adaptive integration. With collisions: integrate until a step ends in
// contact; find the first contact time in that step by bisection on the step length (each trial an
// adaptive integration from the step's start, halving until the interval cannot be split, at most
// 80 times); merge
// the contact pair of lowest member ranks at that time; continue with the merged body. m and R
// (member masses and radii) are updated; ids are the members' body indices (ascending).
template <class T>
static int ce_drift_group(int k, T *y, double *m, const double *rc, const Params &p, double h, double tol,
                          double *R = nullptr, const int64_t *ids = nullptr, MergeCtx *mc = nullptr) {
  const int D = 6 * k;
  std::vector<char> alive_c(k, 1);
  bool *alive = reinterpret_cast<bool *>(alive_c.data());
  const double *Rc = mc ? R : nullptr;
  T t = T(0);
  const T hT = T(h);
  std::vector<T> y0(D), ym(D);
  while (true) {
    T done = T(0), Hc = T(0);
    const int st = gbs_advance<T>(k, y, m, rc, alive, Rc, p, hT - t, tol, mc ? mc->f : 0.0, &done, &Hc);
    if (st == 2) return 1;
    if (st == 0) break;
    t = t + done;
    for (int i = 0; i < D; i++) y0[i] = y[i];
    T lo = T(0), hi = Hc;
    for (int it = 0; it < kMaxBisections; it++) {
      const T mid = (lo + hi) / T(2);
      if (!(val(mid) > val(lo) && val(mid) < val(hi))) break;
      for (int i = 0; i < D; i++) ym[i] = y0[i];
      T d2, h2;
      if (gbs_advance<T>(k, ym.data(), m, rc, alive, nullptr, p, mid, tol, 0.0, &d2, &h2) == 2) return 1;
      if (contact_pair<T>(k, ym.data(), R, alive, mc->f) >= 0) hi = mid; else lo = mid;
    }
    T d2, h2;
    if (gbs_advance<T>(k, y, m, rc, alive, nullptr, p, hi, tol, 0.0, &d2, &h2) == 2) return 1;
    t = t + hi;
    const int pr = contact_pair<T>(k, y, R, alive, mc->f);
    if (pr >= 0) {
      const int a = pr / k, b = pr % k;
      const double M = m[a] + m[b];
      for (int l = 0; l < 3; l++) {
        y[3 * a + l] = (T(m[a]) * y[3 * a + l] + T(m[b]) * y[3 * b + l]) / T(M);
        y[3 * k + 3 * a + l] = (T(m[a]) * y[3 * k + 3 * a + l] + T(m[b]) * y[3 * k + 3 * b + l]) / T(M);
      }
      const double th = 2.0 * M_PI * (double)ids[b] / (double)mc->n;
      const double vc = std::sqrt(p.G * p.m0 / kParkRadius);
      y[3 * b] = T(kParkRadius * std::cos(th));
      y[3 * b + 1] = T(kParkRadius * std::sin(th));
      y[3 * b + 2] = T(0);
      y[3 * k + 3 * b] = T(-vc * std::sin(th));
      y[3 * k + 3 * b + 1] = T(vc * std::cos(th));
      y[3 * k + 3 * b + 2] = T(0);
      R[a] = std::cbrt(R[a] * R[a] * R[a] + R[b] * R[b] * R[b]);
      R[b] = 0.0;
      m[a] = M;
      m[b] = 0.0;
      alive[b] = false;
      mc->log->insert(mc->log->end(), {(int64_t)mc->step, ids[a], ids[b]});
      mc->time->push_back(t);
    }
    if (val(mabs(hT - t)) <= 0) break;
  }
  return 0;
}

// Drift of every body over h with the close-encounter groups given by labels (smallest index of
// each body's group; a body alone in its group keeps the Kepler drift). With mc, bodies of a group
// that come into contact merge (m and R updated). rc holds the critical radii level by level
// ([p.nl][n]); with a mask only the bodies it marks move.
template <class T>
static int drift_groups(int64_t n, T *x, T *v, double *m, const double *rc, const int32_t *label,
                        const Params &p, double h, double tol, int64_t *stats, double *R = nullptr,
                        MergeCtx *mc = nullptr, const char *mask = nullptr) {
  std::vector<std::vector<int64_t>> members((size_t)n);
  for (int64_t i = 0; i < n; i++)
    if (!mask || mask[i]) members[(size_t)label[i]].push_back(i);
  int worst = 0;
  for (int64_t r = 0; r < n; r++) {
    const auto &g = members[(size_t)r];
    if (g.empty()) continue;
    if (g.size() == 1) {
      const int64_t i = g[0];
      worst = std::max(worst, kepler<T>(x + 3 * i, v + 3 * i, p.G * p.m0, h));
      continue;
    }
    const int k = (int)g.size();
    std::vector<T> y(6 * (size_t)k);
    std::vector<double> mg(k), rcg((size_t)p.nl * k), Rg(k, 0.0);
    for (int a = 0; a < k; a++) {
      for (int l = 0; l < 3; l++) {
        y[3 * a + l] = x[3 * g[a] + l];
        y[3 * k + 3 * a + l] = v[3 * g[a] + l];
      }
      mg[a] = m[g[a]];
      for (int l = 0; l < p.nl; l++) rcg[(size_t)l * k + a] = rc[(size_t)l * n + g[a]];
      if (R) Rg[a] = R[g[a]];
    }
    const int st = ce_drift_group<T>(k, y.data(), mg.data(), rcg.data(), p, h, tol, Rg.data(), g.data(), mc);
    worst = std::max(worst, st);
    for (int a = 0; a < k; a++) {
      for (int l = 0; l < 3; l++) {
        x[3 * g[a] + l] = y[3 * a + l];
        v[3 * g[a] + l] = y[3 * k + 3 * a + l];
      }
      if (mc) {
        m[g[a]] = mg[a];
        R[g[a]] = Rg[a];
      }
    }
    if (stats) {
      stats[0] += 1;
      stats[1] = std::max<int64_t>(stats[1], k);
      stats[2] += k;
    }
  }
  return worst;
}

// ---------------------------------------------------------------- multi-level changeover
// Intermediate levels between the symplectic step and the direct integrator (the paper's
// multi-level changeover). Level l has the time step dt_l = dt / s^l and critical radii from
// eq. rcrit at that step, rc_l = max(n1 R_Hill, n2 dt_l v) with the exact-predicate thresholds
// H, V_l. The drift of the bodies in close pairs (the step's level-0 list P0) integrates
// H_A = Kepler + W_0 U, U = -G m_i m_j / r over P0 and W_l = prod_{i <= l} [1 - K_i]. Above the
// deepest level L, a level-l drift over tau is split into s substeps of
//   kick(tau/2s) drift_{l+1}(tau/s) kick(tau/2s),
// where the kick acts on the pairs of P0 with the potential W_l K_{l+1} U and drift_{l+1}
// integrates Kepler + W_{l+1} U. At level L the pairs of P0 closer than rc_L (exact predicate at
// the current positions) form groups integrated with the Gragg-Bulirsch-Stoer method on
// Kepler + W_L U; the other bodies of P0 follow Kepler orbits. Without intermediate levels (L = 0)
// this is the drift of the hybrid step.
struct Levels {
  int L, s;
  int64_t n;
  std::vector<double> rc, H, V;   // [L + 1][n], level-major
};

// Kick over the pairs of P0 with the level-l potential W_{l-1} K_l U (l >= 1), in pair order.
template <class T>
static void level_kick(int64_t n, const T *x, T *v, const double *m, const int32_t *P0, int64_t np,
                       const Levels &lv, int l, const Params &p, T h) {
  std::vector<T> a(3 * (size_t)n, T(0));
  double rcs[8];
  for (int64_t e = 0; e < np; e++) {
    const int64_t i = P0[2 * e], j = P0[2 * e + 1];
    T d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
    T q2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    T q = msqrt(q2);
    for (int k = 0; k <= l; k++) rcs[k] = std::max(lv.rc[(size_t)k * n + i], lv.rc[(size_t)k * n + j]);
    T W, dW, K, dKdy;
    level_weight(q, rcs, l, p, &W, &dW);
    const T span = T((1.0 - p.f_in) * rcs[l]);
    changeover((q - T(p.f_in * rcs[l])) / span, &K, &dKdy);
    const T dK = dKdy / span;
    const T Vw = W * K, dV = dW * K + W * dK;
    const T c = T(p.G) * (Vw / (q2 * q) - dV / q2);
    for (int k = 0; k < 3; k++) {
      a[3 * i + k] = a[3 * i + k] + c * T(m[j]) * d[k];
      a[3 * j + k] = a[3 * j + k] - c * T(m[i]) * d[k];
    }
  }
  for (int64_t i = 0; i < 3 * n; i++) v[i] = v[i] + h * a[i];
}

template <class T>
static int drift_levels(int64_t n, T *x, T *v, double *m, const int32_t *P0, int64_t np,
                        const std::vector<char> &inP0, const Levels &lv, const Params &p, int l, double tau,
                        double tol, int64_t *stats, double *R, MergeCtx *mc) {
  if (l == lv.L) {
    // groups of the level-L close pairs at the current positions
    std::vector<int32_t> PL;
    for (int64_t e = 0; e < np; e++) {
      const int64_t i = P0[2 * e], j = P0[2 * e + 1];
      const double xi[3] = {(double)val(x[3 * i]), (double)val(x[3 * i + 1]), (double)val(x[3 * i + 2])};
      const double xj[3] = {(double)val(x[3 * j]), (double)val(x[3 * j + 1]), (double)val(x[3 * j + 2])};
      double r2;
      const size_t o = (size_t)l * n;
      if (l == 0 || close_pair(xi, xj, lv.H[o + i], lv.H[o + j], lv.V[o + i], lv.V[o + j], &r2)) {
        PL.push_back((int32_t)i);
        PL.push_back((int32_t)j);
      }
    }
    std::vector<int32_t> label(n);
    groups_bfs(n, PL.data(), (int64_t)PL.size() / 2, label.data(), nullptr);
    Params pl = p;
    pl.nl = l + 1;
    return drift_groups<T>(n, x, v, m, lv.rc.data(), label.data(), pl, tau, tol, stats, R, mc, inP0.data());
  }
  const double ts = tau / lv.s;
  int worst = 0;
  for (int k = 0; k < lv.s; k++) {
    level_kick<T>(n, x, v, m, P0, np, lv, l + 1, p, T(0.5 * ts));
    worst = std::max(worst, drift_levels<T>(n, x, v, m, P0, np, inP0, lv, p, l + 1, ts, tol, stats, R, mc));
    level_kick<T>(n, x, v, m, P0, np, lv, l + 1, p, T(0.5 * ts));
  }
  return worst;
}

// nsteps hybrid steps: as steps() but the drift integrates H_A in full, every close-encounter
// group (from the close pairs at the positions of the step's first kick) with ce_drift_group;
// with mc, contacts within a group merge (m and R updated, mergers logged with their step).
// With lv (L > 0), the drift of the bodies in close pairs runs through the intermediate levels.
static int steps_hybrid(int64_t n, double *x, double *v, double *m, const Params &p, int nsteps,
                        const double *rc, const double *H, const double *V, double tol, int64_t *stats,
                        double *R = nullptr, MergeCtx *mc = nullptr, const Levels *lv = nullptr) {
  std::vector<double> acc(3 * n);
  std::vector<int32_t> label(n);
  const double h = 0.5 * p.dt;
  int worst = 0;
  for (int s = 0; s < nsteps; s++) {
    kick_acc<double>(n, x, m, rc, H, V, p, acc.data(), nullptr, nullptr);
    for (int64_t i = 0; i < 3 * n; i++) v[i] = v[i] + h * acc[i];
    const int64_t np = encounters(n, x, H, V, 0, nullptr);
    std::vector<int32_t> pairs(2 * (size_t)std::max<int64_t>(np, 1));
    encounters(n, x, H, V, np, pairs.data());
    groups_bfs(n, pairs.data(), np, label.data(), nullptr);
    jump<double>(n, x, v, m, p, h);
    std::vector<long double> xl(x, x + 3 * n), vl(v, v + 3 * n);
    if (mc) mc->step = s;
    if (lv && lv->L > 0) {
      std::vector<char> inP0(n, 0);
      for (int64_t e = 0; e < np; e++) inP0[pairs[2 * e]] = inP0[pairs[2 * e + 1]] = 1;
      for (int64_t i = 0; i < n; i++)
        if (!inP0[i]) worst = std::max(worst, kepler<long double>(&xl[3 * i], &vl[3 * i], p.G * p.m0, p.dt));
      worst = std::max(worst, drift_levels<long double>(n, xl.data(), vl.data(), m, pairs.data(), np, inP0, *lv,
                                                        p, 0, p.dt, tol, stats, R, mc));
    } else {
      worst = std::max(worst, drift_groups<long double>(n, xl.data(), vl.data(), m, rc, label.data(), p, p.dt,
                                                        tol, stats, R, mc));
    }
    for (int64_t i = 0; i < 3 * n; i++) { x[i] = (double)xl[i]; v[i] = (double)vl[i]; }
    jump<double>(n, x, v, m, p, h);
    kick_acc<double>(n, x, m, rc, H, V, p, acc.data(), nullptr, nullptr);
    for (int64_t i = 0; i < 3 * n; i++) v[i] = v[i] + h * acc[i];
  }
  return worst;
}

template <class T>
static int steps(int64_t n, T *x, T *v, const T *m, const Params &p, int nsteps,
                 const double *rc, const double *H, const double *V) {
  std::vector<T> acc(3 * n);
  T h = T(0.5 * p.dt);
  int worst = 0;
  for (int s = 0; s < nsteps; s++) {
    kick_acc<T>(n, x, m, rc, H, V, p, acc.data(), nullptr, nullptr);
    for (int64_t i = 0; i < 3 * n; i++) v[i] = v[i] + h * acc[i];
    jump<T>(n, x, v, m, p, h);
    worst = std::max(worst, drift_all<T>(n, x, v, p, p.dt, nullptr));
    jump<T>(n, x, v, m, p, h);
    kick_acc<T>(n, x, m, rc, H, V, p, acc.data(), nullptr, nullptr);
    for (int64_t i = 0; i < 3 * n; i++) v[i] = v[i] + h * acc[i];
  }
  return worst;
}

static void vals(int64_t n3, const dual *a, double *out) { for (int64_t i = 0; i < n3; i++) out[i] = a[i].v; }

}  // namespace orc

using namespace orc;

// ================================================================ C entry points
extern "C" {

// Parameter block shared by all calls: G, m0, dt, n1, n2, f_in.
void or_thresholds(int64_t n, const double *x, const double *v, const double *m,
                   const double *prm, double *rc, double *H, double *V) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  thresholds(n, x, v, m, p, rc, H, V);
}

void or_changeover(double y, double *K, double *dKdy) { changeover<double>(y, K, dKdy); }
void or_changeover_q(double y, double *K, double *dKdy) {
  quad k, d;
  changeover<quad>(quad(y), &k, &d);
  *K = (double)k; *dKdy = (double)d;
}

void or_kick_acc(int64_t n, const double *x, const double *m, const double *rc, const double *H,
                 const double *V, const double *prm, double *acc, double *acc_ce, double *l1) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  kick_acc<double>(n, x, m, rc, H, V, p, acc, acc_ce, l1);
}

// The same sum in long double / __float128, rounded to binary64 at the end (accuracy pins).
void or_kick_acc_ld(int64_t n, const double *x, const double *m, const double *rc, const double *H,
                    const double *V, const double *prm, double *acc) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  std::vector<long double> xl(x, x + 3 * n), ml(m, m + n), al(3 * n);
  kick_acc<long double>(n, xl.data(), ml.data(), rc, H, V, p, al.data(), nullptr, nullptr);
  for (int64_t i = 0; i < 3 * n; i++) acc[i] = (double)al[i];
}
void or_kick_acc_q(int64_t n, const double *x, const double *m, const double *rc, const double *H,
                   const double *V, const double *prm, double *acc) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  std::vector<quad> xq(3 * n), mq(n), aq(3 * n);
  for (int64_t i = 0; i < 3 * n; i++) xq[i] = x[i];
  for (int64_t i = 0; i < n; i++) mq[i] = m[i];
  kick_acc<quad>(n, xq.data(), mq.data(), rc, H, V, p, aq.data(), nullptr, nullptr);
  for (int64_t i = 0; i < 3 * n; i++) acc[i] = (double)aq[i];
}

// Accelerations of a subset of bodies (rows idx[0..k)) against all n bodies: lets a test check
// sampled outputs of a large system one by one.
void or_kick_acc_rows(int64_t n, const double *x, const double *m, const double *rc, const double *H,
                      const double *V, const double *prm, int64_t k, const int64_t *idx,
                      double *acc, double *l1) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < k; q++) {
    int64_t i = idx[q];
    Acc<double> a[3];
    double l1s = 0;
    for (int64_t j = 0; j < n; j++) {
      if (j == i) continue;
      double r2d;
      bool close = close_pair(x + 3 * i, x + 3 * j, H[i], H[j], V[i], V[j], &r2d);
      double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
      double w = pair_weight<double>(r2d, close, std::max(rc[i], rc[j]), p.f_in);
      double s = p.G * m[j] * w;
      for (int c = 0; c < 3; c++) a[c].add(s * d[c]);
      l1s += p.G * m[j] * std::fabs(w) * std::sqrt(r2d);
    }
    for (int c = 0; c < 3; c++) acc[3 * q + c] = a[c].get();
    if (l1) l1[q] = l1s;
  }
}

int64_t or_encounters(int64_t n, const double *x, const double *H, const double *V, int64_t cap,
                      int32_t *pairs) {
  return encounters(n, x, H, V, cap, pairs);
}

int64_t or_groups(int64_t n, const int32_t *pairs, int64_t npairs, int32_t *label, int64_t *ignored) {
  return groups_bfs(n, pairs, npairs, label, ignored);
}

// Close-encounter drift of one group (member indices idx[0..k-1] into x, v, m, rc) over time h,
// in long double, to the relative tolerance tol. Returns the integrator status.
int or_ce_drift_group(const int64_t *idx, int k, double *x, double *v, const double *m, const double *rc,
                      const double *prm, double h, double tol) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  std::vector<long double> y(6 * (size_t)k);
  std::vector<double> mg(k), rcg(k);
  for (int a = 0; a < k; a++) {
    for (int l = 0; l < 3; l++) {
      y[3 * a + l] = x[3 * idx[a] + l];
      y[3 * k + 3 * a + l] = v[3 * idx[a] + l];
    }
    mg[a] = m[idx[a]];
    rcg[a] = rc[idx[a]];
  }
  const int st = ce_drift_group<long double>(k, y.data(), mg.data(), rcg.data(), p, h, tol);
  for (int a = 0; a < k; a++)
    for (int l = 0; l < 3; l++) {
      x[3 * idx[a] + l] = (double)y[3 * a + l];
      v[3 * idx[a] + l] = (double)y[3 * k + 3 * a + l];
    }
  return st;
}

// Drift of all bodies over h with the close-encounter groups given by labels (long double;
// stats[3] = {groups integrated, largest group, bodies in groups}, may be NULL).
int or_drift_groups(int64_t n, double *x, double *v, const double *m, const double *rc, const int32_t *label,
                    const double *prm, double h, double tol, int64_t *stats) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  std::vector<long double> xl(x, x + 3 * n), vl(v, v + 3 * n);
  std::vector<double> mm(m, m + n);
  if (stats) stats[0] = stats[1] = stats[2] = 0;
  const int st = drift_groups<long double>(n, xl.data(), vl.data(), mm.data(), rc, label, p, h, tol, stats);
  for (int64_t i = 0; i < 3 * n; i++) { x[i] = (double)xl[i]; v[i] = (double)vl[i]; }
  return st;
}

// Copies a merger log out: up to cap entries of {step, survivor, removed} and their times; returns
// the number of mergers.
static int64_t put_log(const std::vector<int64_t> &log, const std::vector<long double> &time, int64_t cap,
                       int32_t *merges, double *mtime) {
  const int64_t cnt = (int64_t)time.size();
  for (int64_t e = 0; e < std::min(cnt, cap); e++) {
    for (int l = 0; l < 3; l++) merges[3 * e + l] = (int32_t)log[3 * e + l];
    mtime[e] = (double)time[e];
  }
  return cnt;
}

// As or_drift_groups, with collisions: bodies of a group whose distance falls below
// f (R_i + R_j) merge (m and R in/out; mergers logged as {step, survivor, removed} with the time
// within the drift). Returns the integrator status; *count receives the number of mergers.
int or_drift_groups_merge(int64_t n, double *x, double *v, double *m, const double *rc, const int32_t *label,
                          const double *prm, double h, double tol, int64_t *stats, double *R, double f,
                          int step, int32_t *merges, double *mtime, int64_t cap, int64_t *count) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  std::vector<long double> xl(x, x + 3 * n), vl(v, v + 3 * n);
  std::vector<int64_t> log;
  std::vector<long double> time;
  MergeCtx mc{f, n, step, &log, &time};
  if (stats) stats[0] = stats[1] = stats[2] = 0;
  const int st = drift_groups<long double>(n, xl.data(), vl.data(), m, rc, label, p, h, tol, stats, R, &mc);
  for (int64_t i = 0; i < 3 * n; i++) { x[i] = (double)xl[i]; v[i] = (double)vl[i]; }
  *count = put_log(log, time, cap, merges, mtime);
  return st;
}

// nsteps hybrid steps (the drift integrates the close-encounter groups). stats[3] = {groups
// integrated, largest group, bodies in groups}, accumulated over the steps (may be NULL).
int or_step_hybrid(int64_t n, double *x, double *v, const double *m, const double *prm, int nsteps,
                   const double *rc_in, const double *H_in, const double *V_in, double tol, int64_t *stats) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  std::vector<double> rc(n), H(n), V(n);
  if (rc_in && H_in && V_in) {
    std::copy(rc_in, rc_in + n, rc.begin()); std::copy(H_in, H_in + n, H.begin());
    std::copy(V_in, V_in + n, V.begin());
  } else {
    thresholds(n, x, v, m, p, rc.data(), H.data(), V.data());
  }
  if (stats) stats[0] = stats[1] = stats[2] = 0;
  std::vector<double> mm(m, m + n);
  return steps_hybrid(n, x, v, mm.data(), p, nsteps, rc.data(), H.data(), V.data(), tol, stats);
}

// Acceleration of the level-l kick (l >= 1) over the listed pairs: acc = G sum m_j (V/r^3 - V'/r^2) d
// with V = W_{l-1} K_l; rc holds the critical radii of the levels 0..l ([l + 1][n]).
void or_level_kick_acc(int64_t n, const double *x, const double *m, const int32_t *pairs, int64_t np,
                       const double *rc, int l, const double *prm, double *acc) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  Levels lv{l, 1, n, std::vector<double>(rc, rc + (size_t)(l + 1) * n), {}, {}};
  std::vector<double> v(3 * (size_t)n, 0.0);
  level_kick<double>(n, x, v.data(), m, pairs, np, lv, l, p, 1.0);
  std::copy(v.begin(), v.end(), acc);
}

// Close-encounter drift of one group with the pair term weighted by the levels 0..nl-1
// (rc [nl][k] of the members), long double; returns the integrator status.
int or_ce_drift_group_levels(const int64_t *idx, int k, double *x, double *v, const double *m, const double *rc,
                             int nl, const double *prm, double h, double tol) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  p.nl = nl;
  std::vector<long double> y(6 * (size_t)k);
  std::vector<double> mg(k);
  for (int a = 0; a < k; a++) {
    for (int l = 0; l < 3; l++) {
      y[3 * a + l] = x[3 * idx[a] + l];
      y[3 * k + 3 * a + l] = v[3 * idx[a] + l];
    }
    mg[a] = m[idx[a]];
  }
  const int st = ce_drift_group<long double>(k, y.data(), mg.data(), rc, p, h, tol);
  for (int a = 0; a < k; a++)
    for (int l = 0; l < 3; l++) {
      x[3 * idx[a] + l] = (double)y[3 * a + l];
      v[3 * idx[a] + l] = (double)y[3 * k + 3 * a + l];
    }
  return st;
}

// The drift A(h) alone with L intermediate levels (substep factor sub), long double: the bodies
// without listed pairs follow Kepler orbits, the others go through the levels with the pairs as
// the step's close pairs. rc, H, V: [L + 1][n] level thresholds. Returns the integrator status.
int or_drift_levels(int64_t n, double *x, double *v, const double *m, const int32_t *pairs, int64_t np,
                    const double *rc, const double *H, const double *V, int L, int sub, const double *prm,
                    double h, double tol) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  Levels lv{L, sub, n, std::vector<double>(rc, rc + (size_t)(L + 1) * n),
            std::vector<double>(H, H + (size_t)(L + 1) * n), std::vector<double>(V, V + (size_t)(L + 1) * n)};
  std::vector<long double> xl(x, x + 3 * n), vl(v, v + 3 * n);
  std::vector<double> mm(m, m + n);
  std::vector<char> inP0(n, 0);
  for (int64_t e = 0; e < np; e++) inP0[pairs[2 * e]] = inP0[pairs[2 * e + 1]] = 1;
  int worst = 0;
  for (int64_t i = 0; i < n; i++)
    if (!inP0[i]) worst = std::max(worst, kepler<long double>(&xl[3 * i], &vl[3 * i], p.G * p.m0, h));
  worst = std::max(worst, drift_levels<long double>(n, xl.data(), vl.data(), mm.data(), pairs, np, inP0, lv, p, 0,
                                                    h, tol, nullptr, nullptr, nullptr));
  for (int64_t i = 0; i < 3 * n; i++) { x[i] = (double)xl[i]; v[i] = (double)vl[i]; }
  return worst;
}

// nsteps hybrid steps with L intermediate changeover levels (time steps dt / s^l) and, when R is
// given, collisions as perfect mergers (radius factor f; m and R in/out, mergers logged). With
// L > 0 and margin > 0 the step's close-pair list (and the kick's close/far decision, which gives
// the same weight beyond rc since K = 1 there) uses the thresholds H (1+margin)^6, V (1+margin)^2,
// so that pairs crossing rc within the step belong to the drift's pairs.
int or_step_levels(int64_t n, double *x, double *v, double *m, const double *prm, int nsteps,
                   const double *rc_in, const double *H_in, const double *V_in, double tol, int64_t *stats,
                   int L, int sub, double *R, double f, int32_t *merges, double *mtime, int64_t cap,
                   int64_t *count, double margin) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  if (L < 0 || L > 4 || sub < 1) return -1;
  Levels lv{L, sub, n, std::vector<double>((size_t)(L + 1) * n), std::vector<double>((size_t)(L + 1) * n),
            std::vector<double>((size_t)(L + 1) * n)};
  double dtl = p.dt;
  for (int l = 0; l <= L; l++) {
    Params pl = p;
    pl.dt = dtl;
    const size_t o = (size_t)l * n;
    if (l == 0 && rc_in && H_in && V_in) {
      std::copy(rc_in, rc_in + n, lv.rc.begin()); std::copy(H_in, H_in + n, lv.H.begin());
      std::copy(V_in, V_in + n, lv.V.begin());
    } else {
      thresholds(n, x, v, m, pl, lv.rc.data() + o, lv.H.data() + o, lv.V.data() + o);
    }
    dtl = dtl / sub;
  }
  if (stats) stats[0] = stats[1] = stats[2] = 0;
  std::vector<int64_t> log;
  std::vector<long double> time;
  MergeCtx mc{f, n, 0, &log, &time};
  std::vector<double> Hl(lv.H.begin(), lv.H.begin() + n), Vl(lv.V.begin(), lv.V.begin() + n);
  if (L > 0 && margin > 0) {
    const double g = 1.0 + margin, g2 = g * g, g6 = (g2 * g2) * g2;
    for (int64_t i = 0; i < n; i++) {
      Hl[i] = Hl[i] * g6;
      Vl[i] = Vl[i] * g2;
    }
  }
  const int st = steps_hybrid(n, x, v, m, p, nsteps, lv.rc.data(), Hl.data(), Vl.data(), tol, stats,
                              R, R ? &mc : nullptr, &lv);
  *count = put_log(log, time, cap, merges, mtime);
  return st;
}

// nsteps hybrid steps with collisions (perfect mergers at contact, radius factor f): m and R in/out,
// mergers logged as {step, survivor, removed} with the time within the step's drift.
int or_step_merge(int64_t n, double *x, double *v, double *m, const double *prm, int nsteps,
                  const double *rc_in, const double *H_in, const double *V_in, double tol, int64_t *stats,
                  double *R, double f, int32_t *merges, double *mtime, int64_t cap, int64_t *count) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  std::vector<double> rc(n), H(n), V(n);
  if (rc_in && H_in && V_in) {
    std::copy(rc_in, rc_in + n, rc.begin()); std::copy(H_in, H_in + n, H.begin());
    std::copy(V_in, V_in + n, V.begin());
  } else {
    thresholds(n, x, v, m, p, rc.data(), H.data(), V.data());
  }
  if (stats) stats[0] = stats[1] = stats[2] = 0;
  std::vector<int64_t> log;
  std::vector<long double> time;
  MergeCtx mc{f, n, 0, &log, &time};
  const int st = steps_hybrid(n, x, v, m, p, nsteps, rc.data(), H.data(), V.data(), tol, stats, R, &mc);
  *count = put_log(log, time, cap, merges, mtime);
  return st;
}

void or_jump(int64_t n, double *x, const double *v, const double *m, const double *prm, double h) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  jump<double>(n, x, v, m, p, h);
}

int or_drift(int64_t n, double *x, double *v, const double *prm, double h, uint32_t *status) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  return drift_all<double>(n, x, v, p, h, status);
}

// Kepler drift carried out in __float128 (accuracy pin of the long double drift).
int or_drift_q(int64_t n, double *x, double *v, const double *prm, double h) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  int worst = 0;
  for (int64_t i = 0; i < n; i++) {
    quad xq[3], vq[3];
    for (int k = 0; k < 3; k++) { xq[k] = x[3 * i + k]; vq[k] = v[3 * i + k]; }
    worst = std::max(worst, kepler<quad>(xq, vq, p.G * p.m0, h));
    for (int k = 0; k < 3; k++) { x[3 * i + k] = (double)xq[k]; v[3 * i + k] = (double)vq[k]; }
  }
  return worst;
}

// nsteps full steps. If rc/H/V are NULL they are computed from the initial state.
int or_step(int64_t n, double *x, double *v, const double *m, const double *prm, int nsteps,
            const double *rc_in, const double *H_in, const double *V_in) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  std::vector<double> rc(n), H(n), V(n);
  if (rc_in && H_in && V_in) {
    std::copy(rc_in, rc_in + n, rc.begin()); std::copy(H_in, H_in + n, H.begin());
    std::copy(V_in, V_in + n, V.begin());
  } else {
    thresholds(n, x, v, m, p, rc.data(), H.data(), V.data());
  }
  return steps<double>(n, x, v, m, p, nsteps, rc.data(), H.data(), V.data());
}

// Forward-mode derivative (JVP) of nsteps steps in the direction (dx, dv, dm), thresholds held
// fixed at their values from the undisturbed initial state. Outputs the final state and its
// directional derivative.
int or_step_jvp(int64_t n, const double *x, const double *v, const double *m, const double *dx,
                const double *dv, const double *dm, const double *prm, int nsteps,
                double *x_out, double *v_out, double *dx_out, double *dv_out) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  std::vector<double> rc(n), H(n), V(n);
  thresholds(n, x, v, m, p, rc.data(), H.data(), V.data());
  std::vector<dual> X(3 * n), Vv(3 * n), M(n);
  for (int64_t i = 0; i < 3 * n; i++) { X[i] = dual(x[i], dx ? dx[i] : 0.0); Vv[i] = dual(v[i], dv ? dv[i] : 0.0); }
  for (int64_t i = 0; i < n; i++) M[i] = dual(m[i], dm ? dm[i] : 0.0);
  int st = steps<dual>(n, X.data(), Vv.data(), M.data(), p, nsteps, rc.data(), H.data(), V.data());
  vals(3 * n, X.data(), x_out);
  vals(3 * n, Vv.data(), v_out);
  for (int64_t i = 0; i < 3 * n; i++) { dx_out[i] = X[i].d; dv_out[i] = Vv[i].d; }
  return st;
}

// Forward-mode derivatives of the three parts of a step, for checking reverse-mode code.
// Kick: d(acc) for a change (dx, dm) of positions and masses (thresholds fixed).
void or_kick_jvp(int64_t n, const double *x, const double *m, const double *dx, const double *dm,
                 const double *rc, const double *H, const double *V, const double *prm, double *dacc) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  std::vector<dual> X(3 * n), M(n), A(3 * n);
  for (int64_t i = 0; i < 3 * n; i++) X[i] = dual(x[i], dx[i]);
  for (int64_t i = 0; i < n; i++) M[i] = dual(m[i], dm[i]);
  kick_acc<dual>(n, X.data(), M.data(), rc, H, V, p, A.data(), nullptr, nullptr);
  for (int64_t i = 0; i < 3 * n; i++) dacc[i] = A[i].d;
}

// Drift by h: d(x', v') for a change (dx, dv) of the state before the drift.
void or_drift_jvp(int64_t n, const double *x, const double *v, const double *dx, const double *dv,
                  const double *prm, double h, double *dx_out, double *dv_out) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  for (int64_t i = 0; i < n; i++) {
    Dual<long double> X[3], W[3];
    for (int k = 0; k < 3; k++) {
      X[k] = Dual<long double>((long double)x[3 * i + k], (long double)dx[3 * i + k]);
      W[k] = Dual<long double>((long double)v[3 * i + k], (long double)dv[3 * i + k]);
    }
    kepler<Dual<long double>>(X, W, p.G * p.m0, h);
    for (int k = 0; k < 3; k++) { dx_out[3 * i + k] = (double)X[k].d; dv_out[3 * i + k] = (double)W[k].d; }
  }
}

// Jump by h: d(x') for a change (dx, dv, dm).
void or_jump_jvp(int64_t n, const double *x, const double *v, const double *m, const double *dx,
                 const double *dv, const double *dm, const double *prm, double h, double *dx_out) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  std::vector<dual> X(3 * n), W(3 * n), M(n);
  for (int64_t i = 0; i < 3 * n; i++) { X[i] = dual(x[i], dx[i]); W[i] = dual(v[i], dv[i]); }
  for (int64_t i = 0; i < n; i++) M[i] = dual(m[i], dm[i]);
  jump<dual>(n, X.data(), W.data(), M.data(), p, dual(h));
  for (int64_t i = 0; i < 3 * n; i++) dx_out[i] = X[i].d;
}

// Diagnostics: E (full Newtonian), Eprime (pair term weighted by K, the quantity the
// hot-path step conserves), angular momentum L and total momentum P (barycentric velocities).
void or_energy(int64_t n, const double *x, const double *v, const double *m, const double *prm,
               const double *rc, const double *H, const double *V, double *out /*E, E', L[3], P[3]*/) {
  Params p{prm[0], prm[1], prm[2], prm[3], prm[4], prm[5]};
  Acc<double> kin, sun, pairN, pairK, L[3], P[3];
  for (int64_t i = 0; i < n; i++) {
    const double *xi = x + 3 * i, *vi = v + 3 * i;
    kin.add(0.5 * m[i] * (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]));
    sun.add(-p.G * p.m0 * m[i] / std::sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]));
    L[0].add(m[i] * (xi[1] * vi[2] - xi[2] * vi[1]));
    L[1].add(m[i] * (xi[2] * vi[0] - xi[0] * vi[2]));
    L[2].add(m[i] * (xi[0] * vi[1] - xi[1] * vi[0]));
    for (int k = 0; k < 3; k++) P[k].add(m[i] * vi[k]);
  }
  std::vector<double> eN(n), eK(n);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; i++) {
    Acc<double> aN, aK;
    for (int64_t j = i + 1; j < n; j++) {
      double r2;
      bool close = close_pair(x + 3 * i, x + 3 * j, H[i], H[j], V[i], V[j], &r2);
      double r = std::sqrt(r2);
      double e = -p.G * m[i] * m[j] / r;
      aN.add(e);
      double K = 1, dK;
      if (close) {
        double rcij = std::max(rc[i], rc[j]);
        changeover<double>((r - p.f_in * rcij) / ((1 - p.f_in) * rcij), &K, &dK);
      }
      aK.add(e * K);
    }
    eN[i] = aN.get();
    eK[i] = aK.get();
  }
  for (int64_t i = 0; i < n; i++) { pairN.add(eN[i]); pairK.add(eK[i]); }
  double Pv[3] = {P[0].get(), P[1].get(), P[2].get()};
  double hc = (Pv[0] * Pv[0] + Pv[1] * Pv[1] + Pv[2] * Pv[2]) / (2 * p.m0);
  out[0] = kin.get() + sun.get() + pairN.get() + hc;
  out[1] = kin.get() + sun.get() + pairK.get() + hc;
  for (int k = 0; k < 3; k++) { out[2 + k] = L[k].get(); out[5 + k] = Pv[k]; }
}

int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int k) { omp_set_num_threads(k > 0 ? k : 1); }

}  // extern "C"
