// Plain FP64 CPU oracle for the conservative finite-difference MP5 / global
// Lax-Friedrichs / SSPRK scheme of Porth et al. (2014), "MPI-AMRVAC for Solar
// and Astrophysics", Sect. 2.
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// CPU-baseline leg of the benchmark may load this library.  It shares no
// source with the HIP path and the HIP path never calls it.
//
// It is written to be checked by eye against the paper, not to be fast:
//   * scalar loops, no blocking, no fusion;
//   * every stage evaluates the Shu-Osher sum literally from stored stages;
//   * built with -O2 -ffp-contract=off (no FMA contraction, no fast-math).
//
// Templated on the scalar type: `double` for the forward map and `Dual`
// (value + one tangent) for Jacobian-vector products of the whole time
// integration.  Branches (MP5 limiter, minmod, median, global max) are taken
// on the value part, so a JVP differentiates the branch taken at the forward
// point.
//
// Readings of the paper where it is silent (each also listed in the design
// notes of the repository):
//   R1  c_max is the domain-global maximum over all interior cells of all
//       blocks, per direction d, of |v_d| + c_{f,d}, evaluated on the state
//       that L is applied to (Sect. 2.2 calls it the grid-global maximal
//       characteristic velocity).
//   R2  c_f is the textbook fast-magnetosonic speed along d (Sect. 4.4 names
//       it without a formula); the hydro limit is the sound speed.
//   R3  MP5 uses alpha = 4 and eps = 0 (Suresh & Huynh 1997, cited in
//       Sect. 2.2).
//   R4  dt = CFL / max_blocks sum_d c_max,d / dx_d  (Sect. 4.4 gives the 1D
//       form dt < dx / c_w).
//   R5  SSPRK(5,4) uses the printed table except alpha_50 := 1 - (alpha_52 +
//       alpha_53 + alpha_54) so that each row sums to one.  RK3 is the
//       Gottlieb-Shu scheme (cited, not printed, in Sect. 2.3).
//   R6  d|v|/dv := 0 at v = 0 (the derivative a central difference sees).
//       Ties: minmod / min / max take the first argument, the median takes
//       f^L when it equals a bound, the global max keeps the lowest
//       (block, cell) index.
//   R7  LIM03 (Cada & Torrilhon 2009, offered beside MP5 in Sect. 2.2) is
//       their compact third-order function with the asymptotic-region
//       switch: with dm = f_j - f_{j-1}, dp = f_{j+1} - f_j, theta = dm/dp
//       and eta = (dm^2 + dp^2) / (r dx)^2, the interface value is
//       f_j + H/2 with
//         H = (2 dp + dm)/3                       if eta <= 1 (unlimited),
//         H = phi(theta) dp                       otherwise, where
//         phi(theta) = max(0, min(phi3, max(-theta/2, min(2 theta, phi3, 1.6)))),
//         phi3 = (2 + theta)/3,
//       and H = 0 when eta > 1 and dp = 0 (the limit of both one-sided
//       branches).  The radius is r = 1; the switch is sharp (the published
//       smoothing band of width 2 epsilon around eta = 1 is taken with
//       epsilon -> 0).  Sect. 4.5.1 reports third order in both norms for
//       RK3 + LIM03 on the Alfven wave: the limited function alone does not
//       reach it at smooth extrema, and r = 1 does at the resolutions of
//       that test (smaller radii only asymptotically).
//   R8  GLM (Sect. 4.2, the glm3 variant: psi as a ninth variable with flux
//       psi on B_d and c_h^2 B_d on psi, no other psi or div B source terms):
//       the cleaning speed c_h is the largest per-direction c_max of the
//       state L is applied to, and every direction then uses c_h as its
//       c_max, both in the Lax-Friedrichs split (it must bound the +-c_h
//       waves of the psi-B_d subsystem) and in the time step.  The psi decay
//       is operator split after each step: psi *= exp(-dt c_h / c_r) with
//       c_h of the step's initial state and c_r = c_p^2 / c_h = 0.18
//       (the second of the two ways the section names).
//   R9  Hall MHD (Sect. 4.4, conservative Hall MHD in finite differences,
//       with B0 = 0 and eta = 0): the cell-centred current J = curl B by
//       fourth-order central differences along each active direction (an
//       inactive direction contributes no derivative); J of halo cells is
//       the face neighbour's J, so every face must have a neighbour (fixed
//       faces are refused).  Flux terms (eta_h/rho)(B_d J - J_d B) on B and
//       (eta_h/rho)((J.B) B_d - B^2 J_d) on E.  Speed |v_d| + max(c_f,d,
//       eta_h |B| k_max / rho) with k_max = pi max_d 1/dx_d of the cell's
//       block, in the split and in the time step.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <array>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

// Fingerprint of every branch decision taken (MP5 branch, median choice,
// c_max argmax), used by tests to certify that two nearby forward runs took
// the same branches ("non-kinked") before comparing them with a difference
// quotient.  Collected only when enabled (single-threaded runs).
static bool g_hash_on = false;
static uint64_t g_hash = 1469598103934665603ull;
static inline void hash_mix(uint64_t x) {
  if (!g_hash_on) return;
  g_hash ^= x + 0x9e3779b97f4a7c15ull + (g_hash << 6) + (g_hash >> 2);
}

// Operation counter (for the roofline figures of the measurement, not for
// results): Counted is a scalar that counts its arithmetic (+, -, *, /, sqrt,
// exp: one operation each; the oracle forms no fused multiply-add) into the
// current category, and count_cmp counts the comparisons and selections of
// min, max, minmod, median, |x| and the tests that pick a branch.  Units
// (flux evaluations, reconstructions, cells) are counted per category so
// that per-unit averages can be formed.  Enabled by orc_count_ops only
// (single-threaded); otherwise every hook is a no-op.
enum { CAT_OTHER = 0, CAT_FLUX = 1, CAT_RECON = 2, CAT_DIFF = 3, CAT_CMAX = 4, CAT_STAGE = 5, NCAT = 6 };
static bool g_count_on = false;
static int g_cat = CAT_OTHER;
static uint64_t g_nops[NCAT], g_ncmp[NCAT], g_units[NCAT];
static inline void count_cmp(int k = 1) {
  if (g_count_on) g_ncmp[g_cat] += (uint64_t)k;
}
static inline void count_unit(int cat, uint64_t k = 1) {
  if (g_count_on) g_units[cat] += k;
}
static inline void set_cat(int c) {
  if (g_count_on) g_cat = c;
}
// MP5 without its early exit (the median form: the same value for eps = 0);
// a counting option only.
static bool g_mp5_median = false;

struct Counted {
  double v;
  Counted() : v(0.0) {}
  Counted(double x) : v(x) {}
};
static inline Counted cop(double x) {
  if (g_count_on) ++g_nops[g_cat];
  return Counted(x);
}
static inline Counted operator+(Counted a, Counted b) { return cop(a.v + b.v); }
static inline Counted operator-(Counted a, Counted b) { return cop(a.v - b.v); }
static inline Counted operator-(Counted a) { return Counted(-a.v); }
static inline Counted operator*(Counted a, Counted b) { return cop(a.v * b.v); }
static inline Counted operator/(Counted a, Counted b) { return cop(a.v / b.v); }
static inline Counted& operator+=(Counted& a, Counted b) { a = a + b; return a; }
static inline Counted& operator-=(Counted& a, Counted b) { a = a - b; return a; }
static inline Counted sqrt_(Counted a) { return cop(std::sqrt(a.v)); }
static inline Counted exp_(Counted a) { return cop(std::exp(a.v)); }
static inline double val(Counted a) { return a.v; }
static inline bool finite_(Counted a) { return std::isfinite(a.v); }
static inline Counted absv(Counted x) {
  count_cmp();
  return Counted(std::fabs(x.v));
}

// ---------------------------------------------------------------------------
// Forward-mode dual number: value v and one tangent d.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
static inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
static inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
static inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
static inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
static inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
static inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
static inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
static inline Dual sqrt_(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, s > 0.0 ? a.d / (2.0 * s) : 0.0);
}
static inline double sqrt_(double a) { return std::sqrt(a); }
static inline Dual exp_(Dual a) {
  const double e = std::exp(a.v);
  return Dual(e, e * a.d);
}
static inline double exp_(double a) { return std::exp(a); }
static inline double val(double a) { return a; }
static inline double val(Dual a) { return a.v; }
static inline bool finite_(double a) { return std::isfinite(a); }
static inline bool finite_(Dual a) { return std::isfinite(a.v) && std::isfinite(a.d); }

// Forward-mode dual number with N tangents: the local Jacobians of the
// reverse mode (one tangent per input of a cell's flux or of one
// reconstruction).
template <int N> struct DualN {
  double v;
  double d[N];
  DualN() : v(0.0) { for (int k = 0; k < N; ++k) d[k] = 0.0; }
  DualN(double x) : v(x) { for (int k = 0; k < N; ++k) d[k] = 0.0; }
};
template <int N> static inline DualN<N> operator+(const DualN<N>& a, const DualN<N>& b) {
  DualN<N> r(a.v + b.v);
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N> static inline DualN<N> operator-(const DualN<N>& a, const DualN<N>& b) {
  DualN<N> r(a.v - b.v);
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N> static inline DualN<N> operator-(const DualN<N>& a) {
  DualN<N> r(-a.v);
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N> static inline DualN<N> operator*(const DualN<N>& a, const DualN<N>& b) {
  DualN<N> r(a.v * b.v);
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int N> static inline DualN<N> operator/(const DualN<N>& a, const DualN<N>& b) {
  const double q = a.v / b.v;
  DualN<N> r(q);
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - q * b.d[k]) / b.v;
  return r;
}
template <int N> static inline DualN<N>& operator+=(DualN<N>& a, const DualN<N>& b) { a = a + b; return a; }
template <int N> static inline DualN<N>& operator-=(DualN<N>& a, const DualN<N>& b) { a = a - b; return a; }
template <int N> static inline DualN<N> sqrt_(const DualN<N>& a) {
  const double s = std::sqrt(a.v);
  DualN<N> r(s);
  for (int k = 0; k < N; ++k) r.d[k] = s > 0.0 ? a.d[k] / (2.0 * s) : 0.0;
  return r;
}
template <int N> static inline DualN<N> exp_(const DualN<N>& a) {
  const double e = std::exp(a.v);
  DualN<N> r(e);
  for (int k = 0; k < N; ++k) r.d[k] = e * a.d[k];
  return r;
}
template <int N> static inline double val(const DualN<N>& a) { return a.v; }
template <int N> static inline bool finite_(const DualN<N>& a) {
  bool ok = std::isfinite(a.v);
  for (int k = 0; k < N; ++k) ok = ok && std::isfinite(a.d[k]);
  return ok;
}
template <int N> static inline DualN<N> absv(const DualN<N>& x) {
  if (x.v > 0.0) return x;
  if (x.v < 0.0) return -x;
  return DualN<N>(0.0);
}
template <int N> static inline DualN<N> seed(double x, int k) {
  DualN<N> r(x);
  r.d[k] = 1.0;
  return r;
}

// |x| with derivative sign(x), and 0 at x == 0 (reading R6).
static inline double absv(double x) { return std::fabs(x); }
static inline Dual absv(Dual x) {
  if (x.v > 0.0) return x;
  if (x.v < 0.0) return -x;
  return Dual(0.0, 0.0);
}

// min / max returning the first argument on ties.
template <class T> static inline T min2(T a, T b) {
  count_cmp();
  return (val(b) < val(a)) ? b : a;
}
template <class T> static inline T max2(T a, T b) {
  count_cmp();
  return (val(b) > val(a)) ? b : a;
}
template <class T> static inline T min3(T a, T b, T c) { return min2(min2(a, b), c); }
template <class T> static inline T max3(T a, T b, T c) { return max2(max2(a, b), c); }

// ---------------------------------------------------------------------------
// MP5 reconstruction (Suresh & Huynh 1997; selected in Sect. 2.2).
// ---------------------------------------------------------------------------
static const double MP5_ALPHA = 4.0;

// minmod(x, y): 0 unless x and y share a strict sign, else the argument of
// smaller magnitude (first argument on equal magnitudes).
template <class T> static inline T minmod2(T x, T y) {
  count_cmp(2);   // the sign test and the magnitude comparison
  if (val(x) * val(y) <= 0.0) return T(0.0);
  return (std::fabs(val(y)) < std::fabs(val(x))) ? y : x;
}

// minmod of four: sign * min |.| when all four share a strict sign, else 0.
template <class T> static inline T minmod4(T w, T x, T y, T z) {
  count_cmp(8);   // the common-sign tests
  bool pos = val(w) > 0.0 && val(x) > 0.0 && val(y) > 0.0 && val(z) > 0.0;
  bool neg = val(w) < 0.0 && val(x) < 0.0 && val(y) < 0.0 && val(z) < 0.0;
  if (pos) return min2(min2(min2(w, x), y), z);
  if (neg) return max2(max2(max2(w, x), y), z);
  return T(0.0);
}

// Median of three; x is returned when it equals one of the bounds.
template <class T> static inline T median3(T x, T lo, T hi) {
  count_cmp(2);
  // lo <= hi holds for the MP5 bounds (both bracket the centre value).
  if (val(x) < val(lo)) return lo;
  if (val(x) > val(hi)) return hi;
  return x;
}

// Interface value at j+1/2 from the five values f_{j-2}..f_{j+2}, biased to
// the left (upwind for a positive-speed flux F^+).
template <class T> static T mp5(T a, T b, T c, T d, T e, double eps) {
  // fifth-order linear interface value
  T fL = (T(2.0) * a - T(13.0) * b + T(47.0) * c + T(27.0) * d - T(3.0) * e) / T(60.0);
  if (!g_mp5_median) {
    // monotonicity-preserving bound
    T fMP = c + minmod2(d - c, T(MP5_ALPHA) * (c - b));
    count_cmp();
    if (val((fL - c) * (fL - fMP)) <= eps) {   // linear piece 1: fL
      bool flat = val(a) == val(c) && val(b) == val(c) && val(d) == val(c) && val(e) == val(c);
      hash_mix(flat ? 0 : 1);
      return fL;
    }
  }
  // curvatures at j-1, j, j+1
  T dm = a - T(2.0) * b + c;
  T d0 = b - T(2.0) * c + d;
  T dp = c - T(2.0) * d + e;
  T dM4p = minmod4(T(4.0) * d0 - dp, T(4.0) * dp - d0, d0, dp);   // at j+1/2
  T dM4m = minmod4(T(4.0) * d0 - dm, T(4.0) * dm - d0, d0, dm);   // at j-1/2
  T fUL = c + T(MP5_ALPHA) * (c - b);
  T fAV = T(0.5) * (c + d);
  T fMD = fAV - T(0.5) * dM4p;
  T fLC = c + T(0.5) * (c - b) + T(4.0 / 3.0) * dM4m;
  T fmin = max2(min3(c, d, fMD), min3(c, fUL, fLC));
  T fmax = min2(max3(c, d, fMD), max3(c, fUL, fLC));
  T r = median3(fL, fmin, fmax);
  if (g_hash_on) {
    // identify the linear piece returned: fL, or the candidate that set the
    // active bound (with the minmod4 choice behind fMD / fLC).  An exactly
    // flat stencil gets a code of its own: every piece returns the same
    // value there and the same derivative along directions that keep it
    // flat, while rounding of fL decides which piece is reported.
    uint64_t code = 1;
    bool flat = val(a) == val(c) && val(b) == val(c) && val(d) == val(c) && val(e) == val(c);
    if (flat) {
      code = 0;
    } else if (val(r) != val(fL)) {
      auto which = [&](T x) -> uint64_t {
        if (val(x) == val(c)) return 2;
        if (val(x) == val(d)) return 3;
        if (val(x) == val(fUL)) return 4;
        auto m4 = [](T m, T w, T x1, T y, T z) -> uint64_t {
          return val(m) == 0.0 ? 0 : val(m) == val(w) ? 1 : val(m) == val(x1) ? 2 : val(m) == val(y) ? 3 : 4;
        };
        if (val(x) == val(fMD)) return 8 + m4(dM4p, T(4.0) * d0 - dp, T(4.0) * dp - d0, d0, dp);
        return 16 + m4(dM4m, T(4.0) * d0 - dm, T(4.0) * dm - d0, d0, dm);
      };
      code = (val(r) == val(fmin) ? 32 : 64) + which(r);
    }
    hash_mix(code);
  }
  return r;
}

// ---------------------------------------------------------------------------
// LIM03 reconstruction (Cada & Torrilhon 2009; reading R7).
// ---------------------------------------------------------------------------
static const double LIM03_ALPHA = 0.5;   // slope bound at extrema (theta < 0)
static const double LIM03_BETA = 2.0;    // TVD bound phi <= 2 theta
static const double LIM03_GAMMA = 1.6;   // cap below the TVD bound phi <= 2
static double LIM03_RADIUS = 1.0;        // r of the asymptotic region

// Interface value at j+1/2 from f_{j-1}, f_j, f_{j+1}, biased to the left;
// dx is the cell width along the reconstruction direction.
template <class T> static T lim03(T a, T b, T c, double dx) {
  T dm = b - a;   // f_j - f_{j-1}
  T dp = c - b;   // f_{j+1} - f_j
  const double rdx = LIM03_RADIUS * dx;
  T eta = (dm * dm + dp * dp) / T(rdx * rdx);
  count_cmp();
  if (val(eta) <= 1.0) {   // asymptotic region: third-order formula
    hash_mix(0x45);
    return b + T(0.5) * ((T(2.0) * dp + dm) / T(3.0));
  }
  count_cmp();
  if (val(dp) == 0.0) {
    hash_mix(0x40);
    return b;
  }
  T theta = dm / dp;
  T phi3 = (T(2.0) + theta) / T(3.0);
  T lo = T(-LIM03_ALPHA) * theta;
  T tvd = T(LIM03_BETA) * theta;
  T phi = max2(T(0.0), min2(phi3, max2(lo, min3(tvd, phi3, T(LIM03_GAMMA)))));
  if (g_hash_on) {
    uint64_t code = val(phi) == 0.0 ? 0x40 : val(phi) == val(phi3) ? 0x41 : val(phi) == val(lo) ? 0x42
                  : val(phi) == val(tvd) ? 0x43 : 0x44;
    hash_mix(code);
  }
  return b + T(0.5) * phi * dp;
}

// Reconstruction selected for the following calls (0: MP5, 1: LIM03).
static int g_recon = 0;
// Hall parameter of the following calls (reading R9; 0: ideal MHD).
static double g_eta_h = 0.0;

// ---------------------------------------------------------------------------
// Physics (Sect. 3 hydro with an ideal-gas energy equation; Sect. 4.1 and 4.3
// ideal MHD with B0 = 0, eta = eta_h = 0; Sect. 4.2 glm3 for GLM).  Units
// with magnetic pressure B^2/2.
// Variable order: hydro (rho, m_1..m_ndim, E); MHD (rho, m_x, m_y, m_z, E,
// B_x, B_y, B_z); GLM as MHD, then psi.  Phys::mhd is 0 (hydro), 1 (MHD)
// or 2 (GLM).
// ---------------------------------------------------------------------------
struct Phys {
  int ndim;
  int mhd;
  double gamma;
  double eta_h = 0.0;   // Hall parameter (reading R9); 0: ideal MHD
  int nvar() const { return mhd == 2 ? 9 : mhd ? 8 : 2 + ndim; }
  bool glm() const { return mhd == 2; }
  int ncomp() const { return mhd ? 3 : ndim; }   // momentum components
  int iE() const { return 1 + ncomp(); }
};

// Primitive state: rho, v[0..2], p, B[0..2]; returns false if non-physical.
template <class T> struct Prim {
  T rho, v[3], p, B[3];
};

template <class T>
static bool cons_to_prim(const Phys& ph, const T* u, Prim<T>& w) {
  const int nc = ph.ncomp();
  w.rho = u[0];
  for (int k = 0; k < 3; ++k) { w.v[k] = T(0.0); w.B[k] = T(0.0); }
  for (int k = 0; k < nc; ++k) w.v[k] = u[1 + k] / w.rho;
  T kin(0.0);                                   // m.v
  for (int k = 0; k < nc; ++k) kin += u[1 + k] * w.v[k];
  T E = u[ph.iE()];
  T eint = E - T(0.5) * kin;
  if (ph.mhd) {
    T b2(0.0);
    for (int k = 0; k < 3; ++k) { w.B[k] = u[5 + k]; b2 += w.B[k] * w.B[k]; }
    eint = eint - T(0.5) * b2;
  }
  w.p = T(ph.gamma - 1.0) * eint;
  bool ok = finite_(w.rho) && finite_(w.p) && val(w.rho) > 0.0 && val(w.p) > 0.0;
  for (int k = 0; k < nc; ++k) ok = ok && finite_(u[1 + k]);
  return ok;
}

// Physical flux along direction d (ch: the GLM cleaning speed, unused
// otherwise; J: the cell's current, used with the Hall term).
template <class T>
static void phys_flux(const Phys& ph, int d, const T* u, const Prim<T>& w, T* f, T ch = T(0.0),
                      const T* J = nullptr) {
  const int nc = ph.ncomp();
  const T vd = w.v[d];
  f[0] = u[1 + d];                                           // m_d
  if (!ph.mhd) {
    for (int k = 0; k < nc; ++k) f[1 + k] = u[1 + k] * vd;   // m_k v_d
    f[1 + d] = f[1 + d] + w.p;                               // + p delta_kd
    f[ph.iE()] = vd * (u[ph.iE()] + w.p);                    // v_d (E + p)
    return;
  }
  T b2 = w.B[0] * w.B[0] + w.B[1] * w.B[1] + w.B[2] * w.B[2];
  T ptot = w.p + T(0.5) * b2;
  T Bd = w.B[d];
  T bv = w.B[0] * w.v[0] + w.B[1] * w.v[1] + w.B[2] * w.v[2];
  for (int k = 0; k < 3; ++k) f[1 + k] = u[1 + k] * vd - Bd * w.B[k];
  f[1 + d] = f[1 + d] + ptot;
  f[4] = vd * (u[4] + ptot) - Bd * bv;
  for (int k = 0; k < 3; ++k) f[5 + k] = vd * w.B[k] - Bd * w.v[k];
  if (ph.glm()) {
    f[5 + d] = f[5 + d] + u[8];   // + psi delta_kd (the k = d term above is 0)
    f[8] = ch * ch * Bd;          // c_h^2 B_d
  }
  if (ph.eta_h != 0.0 && J) {     // Hall terms (reading R9)
    T h = T(ph.eta_h) / w.rho;
    T jb = J[0] * w.B[0] + J[1] * w.B[1] + J[2] * w.B[2];
    for (int k = 0; k < 3; ++k) f[5 + k] = f[5 + k] + h * (Bd * J[k] - J[d] * w.B[k]);
    f[4] = f[4] + h * (jb * Bd - b2 * J[d]);
  }
}

// GLM: c_r = c_p^2 / c_h of the psi decay (reading R8).
static double GLM_CR = 0.18;

// Fast speed along d (sound speed for hydro).
template <class T>
static T fast_speed(const Phys& ph, int d, const Prim<T>& w) {
  T a2 = T(ph.gamma) * w.p / w.rho;
  if (!ph.mhd) return sqrt_(a2);
  T b2 = (w.B[0] * w.B[0] + w.B[1] * w.B[1] + w.B[2] * w.B[2]) / w.rho;
  T bd2 = w.B[d] * w.B[d] / w.rho;
  T s = a2 + b2;
  T disc = s * s - T(4.0) * a2 * bd2;
  count_cmp();
  if (val(disc) < 0.0) disc = T(0.0);   // rounding guard; >= 0 analytically
  T cf2 = T(0.5) * (s + sqrt_(disc));
  return sqrt_(cf2);
}

// ---------------------------------------------------------------------------
// SSPRK tables in Shu-Osher form (Sect. 2.3).
// ---------------------------------------------------------------------------
struct Scheme {
  int s;
  double alpha[6][6];
  double beta[6][6];
};

static Scheme make_scheme(int id) {
  Scheme S;
  std::memset(&S, 0, sizeof(S));
  if (id == 0) {            // RK3, Gottlieb & Shu (1998)
    S.s = 3;
    S.alpha[1][0] = 1.0;       S.beta[1][0] = 1.0;
    S.alpha[2][0] = 0.75;      S.alpha[2][1] = 0.25; S.beta[2][1] = 0.25;
    S.alpha[3][0] = 1.0 / 3.0; S.alpha[3][2] = 2.0 / 3.0; S.beta[3][2] = 2.0 / 3.0;
  } else if (id == 1) {     // SSPRK(4,3), Sect. 2.3.1
    S.s = 4;
    S.alpha[1][0] = 1.0;       S.beta[1][0] = 0.5;
    S.alpha[2][1] = 1.0;       S.beta[2][1] = 0.5;
    S.alpha[3][0] = 2.0 / 3.0; S.alpha[3][2] = 1.0 / 3.0; S.beta[3][2] = 1.0 / 6.0;
    S.alpha[4][3] = 1.0;       S.beta[4][3] = 0.5;
  } else {                  // SSPRK(5,4), Sect. 2.3.2 (printed digits)
    S.s = 5;
    S.alpha[1][0] = 1.0;
    S.alpha[2][0] = 0.44437049406734; S.alpha[2][1] = 0.55562950593266;
    S.alpha[3][0] = 0.62010185138540; S.alpha[3][2] = 0.37989814861460;
    S.alpha[4][0] = 0.17807995410773; S.alpha[4][3] = 0.82192004589227;
    S.alpha[5][2] = 0.51723167208978; S.alpha[5][3] = 0.12759831133288;
    S.alpha[5][4] = 0.34833675773694;
    // reading R5: the row sum is restored to one through alpha_50
    S.alpha[5][0] = 1.0 - (S.alpha[5][2] + S.alpha[5][3] + S.alpha[5][4]);
    S.beta[1][0] = 0.39175222700392;
    S.beta[2][1] = 0.36841059262959;
    S.beta[3][2] = 0.25189177424738;
    S.beta[4][3] = 0.54497475021237;
    S.beta[5][3] = 0.08460416338212;
    S.beta[5][4] = 0.22600748319395;
  }
  return S;
}

// ---------------------------------------------------------------------------
// Blocks: cell-centred point values with 3 ghost layers in every active
// direction; storage var-major, x fastest (the layout of the public API).
// ---------------------------------------------------------------------------
static const int NG = 3;

struct Geom {
  int n[3];        // interior cells (1 for inactive directions)
  int P[3];        // padded extent
  int G[3];        // ghost depth (3 or 0)
  double dx[3];
  int nbr[6];
  size_t ncell;    // padded cells per variable
  size_t idx(int i, int j, int k) const {
    return ((size_t)(k + G[2]) * P[1] + (size_t)(j + G[1])) * P[0] + (size_t)(i + G[0]);
  }
};

struct Grid {
  Phys ph;
  std::vector<Geom> g;
  // dynamic grid activation (appendix "Dynamic grid activation"): only
  // active blocks are advanced; passive blocks keep their state, which
  // active neighbours read as ghost values.  Empty: every block is active.
  std::vector<unsigned char> active;
  bool is_active(size_t b) const { return active.empty() || active[b] != 0; }
};

// Active flags for the next calls (set by orc_set_active; test infrastructure).
static std::vector<unsigned char> g_active;

template <class T> using State = std::vector<std::vector<T>>;   // [block][var*ncell + idx]

enum { ORC_OK = 0, ORC_ERR_INVALID = 1, ORC_ERR_NONPHYSICAL = 4 };

static int build_grid(Grid& G, int ndim, int mhd, double gamma, int nb, const int* n,
                      const double* dx, const int* nbr) {
  if (ndim < 1 || ndim > 3 || nb <= 0 || mhd < 0 || mhd > 2) return ORC_ERR_INVALID;
  G.ph.ndim = ndim; G.ph.mhd = mhd; G.ph.gamma = gamma;
  G.ph.eta_h = (mhd == 1) ? g_eta_h : 0.0;
  G.g.resize(nb);
  for (int b = 0; b < nb; ++b) {
    Geom& q = G.g[b];
    for (int d = 0; d < 3; ++d) {
      bool act = d < ndim;
      q.n[d] = act ? n[3 * b + d] : 1;
      if (act && q.n[d] < NG) return ORC_ERR_INVALID;
      q.G[d] = act ? NG : 0;
      q.P[d] = q.n[d] + 2 * q.G[d];
      q.dx[d] = dx[3 * b + d];
    }
    for (int f = 0; f < 6; ++f) q.nbr[f] = (f < 2 * ndim) ? nbr[6 * b + f] : -1;
    q.ncell = (size_t)q.P[0] * q.P[1] * q.P[2];
  }
  G.active.clear();
  if ((int)g_active.size() == nb) G.active = g_active;
  return ORC_OK;
}

// Copy the 3 face layers of every periodic (nbr >= 0) face from the
// neighbour's interior; fixed faces (nbr < 0) keep their values.  Edges and
// corners are never read by the dimension-by-dimension operator.
template <class T>
static void fill_ghosts(const Grid& G, State<T>& U, int nv_override = 0) {
  const int nv = nv_override > 0 ? nv_override : G.ph.nvar();
  for (size_t b = 0; b < G.g.size(); ++b) {
    const Geom& q = G.g[b];
    for (int d = 0; d < G.ph.ndim; ++d) {
      for (int side = 0; side < 2; ++side) {
        int nb = q.nbr[2 * d + side];
        if (nb < 0) continue;
        const Geom& r = G.g[nb];
        for (int layer = 1; layer <= NG; ++layer) {
          int dst = side == 0 ? -layer : q.n[d] - 1 + layer;       // ghost index along d
          int src = side == 0 ? r.n[d] - layer : layer - 1;        // neighbour interior
          int lo[3] = {0, 0, 0}, hi[3] = {q.n[0], q.n[1], q.n[2]};
          lo[d] = 0; hi[d] = 1;
          for (int k = lo[2]; k < hi[2]; ++k)
            for (int j = lo[1]; j < hi[1]; ++j)
              for (int i = lo[0]; i < hi[0]; ++i) {
                int cd[3] = {i, j, k}, cs[3] = {i, j, k};
                cd[d] = dst; cs[d] = src;
                for (int v = 0; v < nv; ++v)
                  U[b][v * q.ncell + q.idx(cd[0], cd[1], cd[2])] =
                      U[nb][v * r.ncell + r.idx(cs[0], cs[1], cs[2])];
              }
        }
      }
    }
  }
}

// Domain-global per-direction maximum of |v_d| + c_{f,d} over interior
// cells (reading R1).  Ties keep the first (lowest block, lowest cell).
template <class T>
static int global_cmax(const Grid& G, const State<T>& U, T cmax[3], uint64_t* argout = nullptr) {
  const int nv = G.ph.nvar();
  for (int d = 0; d < 3; ++d) cmax[d] = T(0.0);
  uint64_t arg[3] = {0, 0, 0};
  bool first = true;
  for (size_t b = 0; b < G.g.size(); ++b) {
    if (!G.is_active(b)) continue;
    const Geom& q = G.g[b];
    for (int k = 0; k < q.n[2]; ++k)
      for (int j = 0; j < q.n[1]; ++j)
        for (int i = 0; i < q.n[0]; ++i) {
          T u[9];
          size_t c = q.idx(i, j, k);
          for (int v = 0; v < nv; ++v) u[v] = U[b][v * q.ncell + c];
          set_cat(CAT_CMAX);
          count_unit(CAT_CMAX);
          Prim<T> w;
          if (!cons_to_prim(G.ph, u, w)) return ORC_ERR_NONPHYSICAL;
          for (int d = 0; d < G.ph.ndim; ++d) {
            T cf = fast_speed(G.ph, d, w);
            if (G.ph.eta_h != 0.0) {   // fast whistler at k_max (reading R9)
              double kmax = 0.0;
              for (int e = 0; e < G.ph.ndim; ++e) kmax = std::max(kmax, 1.0 / q.dx[e]);
              kmax = M_PI * kmax;
              T babs = sqrt_(w.B[0] * w.B[0] + w.B[1] * w.B[1] + w.B[2] * w.B[2]);
              T wh = T(G.ph.eta_h) * babs / w.rho * T(kmax);
              if (val(wh) > val(cf)) cf = wh;
            }
            T s = absv(w.v[d]) + cf;
            count_cmp();
            if (first || val(s) > val(cmax[d])) { cmax[d] = s; arg[d] = ((uint64_t)b << 32) | c; }
          }
          first = false;
        }
  }
  for (int d = 0; d < G.ph.ndim; ++d) hash_mix(arg[d] * 3 + d);
  if (argout)
    for (int d = 0; d < 3; ++d) argout[d] = arg[d];
  if (G.ph.glm()) {   // reading R8: c_h = max_d c_max,d for every direction
    T ch = cmax[0];
    for (int d = 1; d < G.ph.ndim; ++d)
      if (val(cmax[d]) > val(ch)) ch = cmax[d];
    for (int d = 0; d < G.ph.ndim; ++d) cmax[d] = ch;
  }
  return ORC_OK;
}

// Right-hand side L(U) = - sum_d (Fhat_{i+1/2} - Fhat_{i-1/2}) / dx_d on the
// interior of every block (Sect. 2.1, eqs. fdcons and timeoperator, S = 0),
// with Fhat from the global Lax-Friedrichs split and MP5 (Sect. 2.2).
// Ghost layers of U must be filled.  L has the padded layout; its ghost
// entries are left at zero.
// Cell-centred current J = curl B (Sect. 4.4, eq. jcd4 at cell centres) on
// the interior cells of every block, then on the halo cells from the face
// neighbours.  U's ghosts must be filled.  Fixed faces are refused.
template <class T>
static int current(const Grid& G, const State<T>& U, State<T>& J) {
  const int nb = (int)G.g.size();
  J.resize(nb);
  for (int b = 0; b < nb; ++b) {
    const Geom& q = G.g[b];
    for (int d = 0; d < G.ph.ndim; ++d)
      if (q.nbr[2 * d] < 0 || q.nbr[2 * d + 1] < 0) return ORC_ERR_INVALID;
    J[b].assign(3 * q.ncell, T(0.0));
    for (int k = 0; k < q.n[2]; ++k)
      for (int j = 0; j < q.n[1]; ++j)
        for (int i = 0; i < q.n[0]; ++i) {
          T dB[3][3];   // dB[a][c] = d B_c / d x_a
          for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
              dB[a][c] = T(0.0);
              if (a >= G.ph.ndim) continue;
              auto Bc = [&](int sft) {
                int p3[3] = {i, j, k};
                p3[a] += sft;
                return U[b][(5 + c) * q.ncell + q.idx(p3[0], p3[1], p3[2])];
              };
              dB[a][c] = (T(-1.0) * Bc(2) + T(8.0) * Bc(1) - T(8.0) * Bc(-1) + Bc(-2)) / T(12.0 * q.dx[a]);
            }
          const size_t o = q.idx(i, j, k);
          J[b][0 * q.ncell + o] = dB[1][2] - dB[2][1];
          J[b][1 * q.ncell + o] = dB[2][0] - dB[0][2];
          J[b][2 * q.ncell + o] = dB[0][1] - dB[1][0];
        }
  }
  fill_ghosts(G, J, 3);
  return ORC_OK;
}

template <class T>
static int rhs(const Grid& G, const State<T>& U, const T cmax[3], State<T>& L, double eps) {
  const int nv = G.ph.nvar();
  const int nb = (int)G.g.size();
  int status = ORC_OK;
  State<T> Jc;
  const bool hall = G.ph.eta_h != 0.0;
  if (hall) {
    int st = current(G, U, Jc);
    if (st) return st;
  }
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < nb; ++b) {
    const Geom& q = G.g[b];
    std::fill(L[b].begin(), L[b].end(), T(0.0));
    if (!G.is_active(b)) continue;
    for (int d = 0; d < G.ph.ndim; ++d) {
      const int nd = q.n[d];
      const int len = nd + 2 * NG;
      std::vector<T> Fp(nv * len), Fm(nv * len), Fh(nv * (nd + 1));
      int lo[3] = {0, 0, 0}, hi[3] = {q.n[0], q.n[1], q.n[2]};
      hi[d] = 1;
      for (int k = lo[2]; k < hi[2]; ++k)
        for (int j = lo[1]; j < hi[1]; ++j)
          for (int i = lo[0]; i < hi[0]; ++i) {
            // split fluxes along the pencil, cells -3 .. nd+2
            set_cat(CAT_FLUX);
            for (int m = -NG; m < nd + NG; ++m) {
              count_unit(CAT_FLUX);
              int c3[3] = {i, j, k};
              c3[d] = m;
              size_t c = q.idx(c3[0], c3[1], c3[2]);
              T u[9], f[9];
              for (int v = 0; v < nv; ++v) u[v] = U[b][v * q.ncell + c];
              Prim<T> w;
              if (!cons_to_prim(G.ph, u, w)) {
#pragma omp atomic write
                status = ORC_ERR_NONPHYSICAL;
              }
              T jc[3] = {T(0.0), T(0.0), T(0.0)};
              if (hall)
                for (int v = 0; v < 3; ++v) jc[v] = Jc[b][v * q.ncell + c];
              phys_flux(G.ph, d, u, w, f, cmax[d], hall ? jc : nullptr);
              for (int v = 0; v < nv; ++v) {
                Fp[v * len + (m + NG)] = T(0.5) * (f[v] + cmax[d] * u[v]);
                Fm[v * len + (m + NG)] = T(0.5) * (f[v] - cmax[d] * u[v]);
              }
            }
            // interface fluxes at i+1/2 for i = -1 .. nd-1
            set_cat(CAT_RECON);
            count_unit(CAT_RECON, 2 * (uint64_t)nv * (nd + 1));
            for (int v = 0; v < nv; ++v) {
              const T* p = &Fp[v * len + NG];
              const T* mneg = &Fm[v * len + NG];
              for (int s = -1; s < nd; ++s) {
                T plus, minus;
                if (g_recon == 1) {
                  plus = lim03(p[s - 1], p[s], p[s + 1], q.dx[d]);
                  minus = lim03(mneg[s + 2], mneg[s + 1], mneg[s], q.dx[d]);
                } else {
                  plus = mp5(p[s - 2], p[s - 1], p[s], p[s + 1], p[s + 2], eps);
                  minus = mp5(mneg[s + 3], mneg[s + 2], mneg[s + 1], mneg[s], mneg[s - 1], eps);
                }
                Fh[v * (nd + 1) + (s + 1)] = plus + minus;
              }
            }
            // conservative difference
            set_cat(CAT_DIFF);
            count_unit(CAT_DIFF, (uint64_t)nv * nd);
            for (int s = 0; s < nd; ++s) {
              int c3[3] = {i, j, k};
              c3[d] = s;
              size_t c = q.idx(c3[0], c3[1], c3[2]);
              for (int v = 0; v < nv; ++v) {
                T diff = Fh[v * (nd + 1) + (s + 1)] - Fh[v * (nd + 1) + s];
                L[b][v * q.ncell + c] -= diff / T(q.dx[d]);
              }
            }
          }
    }
  }
  return status;
}

template <class T>
static void alloc_state(const Grid& G, State<T>& S) {
  S.resize(G.g.size());
  for (size_t b = 0; b < G.g.size(); ++b) S[b].assign(G.ph.nvar() * G.g[b].ncell, T(0.0));
}

static double dt_rule(const Grid& G, const double cmax[3], double cfl) {
  double worst = 0.0;
  for (size_t b = 0; b < G.g.size(); ++b) {
    if (!G.is_active(b)) continue;
    const Geom& q = G.g[b];
    double s = 0.0;
    for (int d = 0; d < G.ph.ndim; ++d) s += cmax[d] / q.dx[d];
    worst = std::max(worst, s);
  }
  return cfl / worst;
}

// One SSPRK step in literal Shu-Osher form:
//   U(0) = U^n,  U(i) = sum_{k<i} alpha_ik U(k) + dt beta_ik L(U(k)),
//   U^{n+1} = U(s)      (Sect. 2.3).
// dt < 0 selects the CFL rule R4 evaluated on U^n; the dt used is returned.
template <class T>
static int ssprk_step(const Grid& G, const Scheme& S, State<T>& U, double cfl, double dt_in,
                      double eps, double* dt_used) {
  const int nv = G.ph.nvar();
  std::vector<State<T>> Us(S.s + 1), Ls(S.s);
  Us[0] = U;
  double dt = dt_in;
  T ch0(0.0);   // GLM cleaning speed of U^n
  for (int i = 1; i <= S.s; ++i) {
    // L(U(i-1)) is the only new right-hand side this stage needs.
    int k = i - 1;
    fill_ghosts(G, Us[k]);
    T cm[3];
    int st = global_cmax(G, Us[k], cm);
    if (st) return st;
    if (k == 0) ch0 = cm[0];
    if (k == 0 && dt_in < 0.0) {
      double cv[3] = {val(cm[0]), val(cm[1]), val(cm[2])};
      dt = dt_rule(G, cv, cfl);
    }
    alloc_state(G, Ls[k]);
    st = rhs(G, Us[k], cm, Ls[k], eps);
    if (st) return st;
    Us[i] = Us[0];   // ghost layers: fixed faces keep U^n's values; passive blocks keep U^n
    set_cat(CAT_STAGE);
    for (size_t b = 0; b < G.g.size(); ++b) {
      if (!G.is_active(b)) continue;
      const Geom& q = G.g[b];
      count_unit(CAT_STAGE, (uint64_t)q.n[0] * q.n[1] * q.n[2]);
      for (int kk = 0; kk < q.n[2]; ++kk)
        for (int j = 0; j < q.n[1]; ++j)
          for (int ii = 0; ii < q.n[0]; ++ii) {
            size_t c = q.idx(ii, j, kk);
            for (int v = 0; v < nv; ++v) {
              size_t o = v * q.ncell + c;
              T acc(0.0);
              for (int m = 0; m < i; ++m) {
                if (S.alpha[i][m] != 0.0) acc += T(S.alpha[i][m]) * Us[m][b][o];
                if (S.beta[i][m] != 0.0) acc += T(dt * S.beta[i][m]) * Ls[m][b][o];
              }
              Us[i][b][o] = acc;
            }
          }
    }
  }
  U = Us[S.s];
  if (G.ph.glm()) {
    // operator-split decay of psi (reading R8), interior cells of active blocks
    T decay = exp_(T(-dt / GLM_CR) * ch0);
    for (size_t b = 0; b < G.g.size(); ++b) {
      if (!G.is_active(b)) continue;
      const Geom& q = G.g[b];
      for (int kk = 0; kk < q.n[2]; ++kk)
        for (int j = 0; j < q.n[1]; ++j)
          for (int ii = 0; ii < q.n[0]; ++ii) {
            size_t o = 8 * q.ncell + q.idx(ii, j, kk);
            U[b][o] = U[b][o] * decay;
          }
    }
  }
  if (dt_used) *dt_used = dt;
  return ORC_OK;
}

// ---------------------------------------------------------------------------
// Reverse mode (adjoint) of the time integration at a fixed dt.
//
// The map differentiated is U^0 -> U^N of the scheme above, with c_max a
// function of every stage state (its derivative goes to the maximising cell)
// and, for fixed faces, the caller's ghost values as further inputs
// (constant in time).  Local Jacobians come from dual numbers through the
// same forward functions (the flux of each cell, each reconstruction), and
// are applied transposed and scattered (no hand-written derivative):
//   L_i = -(Fhat_{i+1/2} - Fhat_{i-1/2}) / dx   (per direction)
//   => lamFhat_{i+1/2} = (mu_{i+1} - mu_i) / dx  (mu = 0 outside the interior)
//   Fhat = R(F+ stencil) + R(F- stencil)
//   => lamF+-_j += lamFhat * dR/dF+-_j           (dual numbers through R)
//   F+-_j = (F(U_j) +- c U_j) / 2
//   => lamU_j += (dF+-/dU_j)^T lamF+-_j,  lam_c += sum_j U_j (lamF+_j - lamF-_j)/2
//   c = |v_d| + c_f,d at the maximising cell
//   => lamU_argmax += lam_c d(|v_d| + c_f,d)/dU
// Adjoints landing on the ghost cells of a periodic face belong to the
// neighbour's interior cell they copy (the transpose of the ghost fill);
// on a fixed face they are the adjoint of the boundary data.
// ---------------------------------------------------------------------------

// lam += scale * (dL/dU)^T mu for the state U (ghosts filled) with c_max
// cmax and maximising cells arg (global_cmax's keys).  lam, gadj: padded
// accumulators; interior entries of lam receive the interior adjoint,
// gadj the fixed faces' ghost entries.
static int rhs_vjp(const Grid& G, const State<double>& U, const double cmax[3], const uint64_t arg[3],
                   const State<double>& mu, double scale, double eps, State<double>& lam, State<double>& gadj) {
  const int nv = G.ph.nvar();
  const int nb = (int)G.g.size();
  State<double> acc(nb);   // per block: padded adjoint of this block's cells (its ghosts included)
  std::vector<double> lamc(3 * nb, 0.0);
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < nb; ++b) {
    const Geom& q = G.g[b];
    acc[b].assign(nv * q.ncell, 0.0);
    for (int d = 0; d < G.ph.ndim; ++d) {
      const int nd = q.n[d];
      const int len = nd + 2 * NG;
      const double c = cmax[d];
      std::vector<double> lp(nv * len), lm(nv * len), Fp(nv * len), Fm(nv * len);
      int lo[3] = {0, 0, 0}, hi[3] = {q.n[0], q.n[1], q.n[2]};
      hi[d] = 1;
      for (int k = lo[2]; k < hi[2]; ++k)
        for (int j = lo[1]; j < hi[1]; ++j)
          for (int i = lo[0]; i < hi[0]; ++i) {
            auto cell = [&](int m) {
              int c3[3] = {i, j, k};
              c3[d] = m;
              return q.idx(c3[0], c3[1], c3[2]);
            };
            // split fluxes along the pencil, cells -3 .. nd+2
            for (int m = -NG; m < nd + NG; ++m) {
              double u[9], f[9];
              const size_t o = cell(m);
              for (int v = 0; v < nv; ++v) u[v] = U[b][v * q.ncell + o];
              Prim<double> w;
              cons_to_prim(G.ph, u, w);
              phys_flux(G.ph, d, u, w, f);
              for (int v = 0; v < nv; ++v) {
                Fp[v * len + m + NG] = 0.5 * (f[v] + c * u[v]);
                Fm[v * len + m + NG] = 0.5 * (f[v] - c * u[v]);
              }
            }
            std::fill(lp.begin(), lp.end(), 0.0);
            std::fill(lm.begin(), lm.end(), 0.0);
            // interfaces s+1/2, s = -1 .. nd-1: lamFhat and the reconstruction
            // weights (dual numbers, one tangent per stencil value)
            for (int v = 0; v < nv; ++v) {
              auto muv = [&](int m) { return (m >= 0 && m < nd) ? mu[b][v * q.ncell + cell(m)] : 0.0; };
              const double* p = &Fp[v * len + NG];
              const double* mneg = &Fm[v * len + NG];
              for (int sI = -1; sI < nd; ++sI) {
                const double lf = (muv(sI + 1) - muv(sI)) / q.dx[d];
                if (lf == 0.0) continue;
                if (g_recon == 1) {
                  DualN<3> a[3], bm[3];
                  for (int t = 0; t < 3; ++t) {
                    a[t] = seed<3>(p[sI - 1 + t], t);
                    bm[t] = seed<3>(mneg[sI + 2 - t], t);
                  }
                  DualN<3> rp = lim03(a[0], a[1], a[2], q.dx[d]);
                  DualN<3> rm = lim03(bm[0], bm[1], bm[2], q.dx[d]);
                  for (int t = 0; t < 3; ++t) {
                    lp[v * len + (sI - 1 + t) + NG] += lf * rp.d[t];
                    lm[v * len + (sI + 2 - t) + NG] += lf * rm.d[t];
                  }
                } else {
                  DualN<5> a[5], bm[5];
                  for (int t = 0; t < 5; ++t) {
                    a[t] = seed<5>(p[sI - 2 + t], t);
                    bm[t] = seed<5>(mneg[sI + 3 - t], t);
                  }
                  DualN<5> rp = mp5(a[0], a[1], a[2], a[3], a[4], eps);
                  DualN<5> rm = mp5(bm[0], bm[1], bm[2], bm[3], bm[4], eps);
                  for (int t = 0; t < 5; ++t) {
                    lp[v * len + (sI - 2 + t) + NG] += lf * rp.d[t];
                    lm[v * len + (sI + 3 - t) + NG] += lf * rm.d[t];
                  }
                }
              }
            }
            // split adjoint: flux Jacobian of each cell by dual numbers
            for (int m = -NG; m < nd + NG; ++m) {
              const size_t o = cell(m);
              bool any = false;
              for (int v = 0; v < nv; ++v) any = any || lp[v * len + m + NG] != 0.0 || lm[v * len + m + NG] != 0.0;
              if (!any) continue;
              DualN<9> u[9], f[9];
              for (int v = 0; v < nv; ++v) u[v] = seed<9>(U[b][v * q.ncell + o], v);
              Prim<DualN<9>> w;
              cons_to_prim(G.ph, u, w);
              phys_flux(G.ph, d, u, w, f);
              for (int t = 0; t < nv; ++t) {
                double g = 0.0;
                for (int v = 0; v < nv; ++v) {
                  const double a = lp[v * len + m + NG], bmv = lm[v * len + m + NG];
                  // d(F+-_v)/dU_t = (dF_v/dU_t +- c delta_vt) / 2
                  g += a * 0.5 * (f[v].d[t] + (v == t ? c : 0.0)) + bmv * 0.5 * (f[v].d[t] - (v == t ? c : 0.0));
                }
                acc[b][t * q.ncell + o] += scale * g;
              }
              for (int v = 0; v < nv; ++v)
                lamc[3 * b + d] += 0.5 * U[b][v * q.ncell + o] * (lp[v * len + m + NG] - lm[v * len + m + NG]);
            }
          }
    }
  }
  // ghost adjoints: periodic faces to the neighbour's interior cell the ghost
  // copies, fixed faces to the boundary-data adjoint
  for (int b = 0; b < nb; ++b) {
    const Geom& q = G.g[b];
    for (int k = -q.G[2]; k < q.n[2] + q.G[2]; ++k)
      for (int j = -q.G[1]; j < q.n[1] + q.G[1]; ++j)
        for (int i = -q.G[0]; i < q.n[0] + q.G[0]; ++i) {
          int c3[3] = {i, j, k};
          int out = 0, od = -1;
          for (int d = 0; d < 3; ++d)
            if (c3[d] < 0 || c3[d] >= q.n[d]) { ++out; od = d; }
          const size_t o = q.idx(i, j, k);
          if (out == 0) {
            for (int v = 0; v < nv; ++v) lam[b][v * q.ncell + o] += acc[b][v * q.ncell + o];
            continue;
          }
          if (out > 1) continue;   // edge and corner ghosts are never read
          const int side = c3[od] < 0 ? 0 : 1;
          const int nbk = q.nbr[2 * od + side];
          if (nbk < 0) {
            for (int v = 0; v < nv; ++v) gadj[b][v * q.ncell + o] += acc[b][v * q.ncell + o];
            continue;
          }
          const Geom& r = G.g[nbk];
          int s3[3] = {i, j, k};
          s3[od] = side == 0 ? c3[od] + r.n[od] : c3[od] - q.n[od];
          const size_t os = r.idx(s3[0], s3[1], s3[2]);
          for (int v = 0; v < nv; ++v) lam[nbk][v * r.ncell + os] += acc[b][v * q.ncell + o];
        }
  }
  // c_max: lam_c (summed over blocks in order) times the derivative of the
  // maximising cell's |v_d| + c_f,d
  for (int d = 0; d < G.ph.ndim; ++d) {
    double lc = 0.0;
    for (int b = 0; b < nb; ++b) lc += lamc[3 * b + d];
    if (lc == 0.0) continue;
    const int b = (int)(arg[d] >> 32);
    const size_t o = (size_t)(arg[d] & 0xffffffffull);
    const Geom& q = G.g[b];
    DualN<9> u[9];
    for (int v = 0; v < nv; ++v) u[v] = seed<9>(U[b][v * q.ncell + o], v);
    Prim<DualN<9>> w;
    if (!cons_to_prim(G.ph, u, w)) return ORC_ERR_NONPHYSICAL;
    DualN<9> sp = absv(w.v[d]) + fast_speed(G.ph, d, w);
    for (int t = 0; t < nv; ++t) lam[b][t * q.ncell + o] += scale * lc * sp.d[t];
  }
  return ORC_OK;
}

// Reverse of one step from U^n (ghosts as given) at fixed dt: lam holds
// dJ/dU^{n+1} on entry (interior) and dJ/dU^n on return; gadj accumulates
// the boundary-data adjoint.  The stage states are recomputed from U^n.
static int ssprk_step_vjp(const Grid& G, const Scheme& S, const State<double>& Un, double dt, double eps,
                          State<double>& lam, State<double>& gadj) {
  const int nv = G.ph.nvar();
  std::vector<State<double>> Us(S.s + 1), Ls(S.s);
  std::vector<std::array<double, 3>> cms(S.s);
  std::vector<std::array<uint64_t, 3>> args(S.s);
  Us[0] = Un;
  for (int i = 1; i <= S.s; ++i) {
    const int k = i - 1;
    fill_ghosts(G, Us[k]);
    double cm[3];
    uint64_t ag[3];
    int st = global_cmax(G, Us[k], cm, ag);
    if (st) return st;
    for (int d = 0; d < 3; ++d) { cms[k][d] = cm[d]; args[k][d] = ag[d]; }
    if (i == S.s) break;   // U(s) is not needed
    alloc_state(G, Ls[k]);
    st = rhs(G, Us[k], cm, Ls[k], eps);
    if (st) return st;
    Us[i] = Us[0];
    for (size_t b = 0; b < G.g.size(); ++b) {
      const Geom& q = G.g[b];
      for (int kk = 0; kk < q.n[2]; ++kk)
        for (int j = 0; j < q.n[1]; ++j)
          for (int ii = 0; ii < q.n[0]; ++ii) {
            const size_t c = q.idx(ii, j, kk);
            for (int v = 0; v < nv; ++v) {
              const size_t o = v * q.ncell + c;
              double a = 0.0;
              for (int m = 0; m < i; ++m) {
                if (S.alpha[i][m] != 0.0) a += S.alpha[i][m] * Us[m][b][o];
                if (S.beta[i][m] != 0.0) a += dt * S.beta[i][m] * Ls[m][b][o];
              }
              Us[i][b][o] = a;
            }
          }
    }
  }
  // lam(s) = lam; lam(k) = sum_{i>k} alpha_ik lam(i) + dt J_L(U(k))^T sum_{i>k} beta_ik lam(i)
  std::vector<State<double>> La(S.s + 1);
  La[S.s] = lam;
  for (int k = S.s - 1; k >= 0; --k) {
    alloc_state(G, La[k]);
    State<double> mu;
    alloc_state(G, mu);
    bool any_mu = false;
    for (size_t b = 0; b < G.g.size(); ++b)
      for (size_t o = 0; o < La[k][b].size(); ++o) {
        double a = 0.0, m = 0.0;
        for (int i = k + 1; i <= S.s; ++i) {
          if (S.alpha[i][k] != 0.0) a += S.alpha[i][k] * La[i][b][o];
          if (S.beta[i][k] != 0.0) m += S.beta[i][k] * La[i][b][o];
        }
        La[k][b][o] = a;
        mu[b][o] = m;
      }
    for (int i = k + 1; i <= S.s; ++i) any_mu = any_mu || S.beta[i][k] != 0.0;
    if (any_mu) {
      const double cm[3] = {cms[k][0], cms[k][1], cms[k][2]};
      const uint64_t ag[3] = {args[k][0], args[k][1], args[k][2]};
      int st = rhs_vjp(G, Us[k], cm, ag, mu, dt, eps, La[k], gadj);
      if (st) return st;
    }
  }
  lam = La[0];
  return ORC_OK;
}

template <class T>
static void load_state(const Grid& G, State<T>& U, const double* const* u) {
  alloc_state(G, U);
  for (size_t b = 0; b < G.g.size(); ++b)
    for (size_t o = 0; o < U[b].size(); ++o) U[b][o] = T(u[b][o]);
}

}  // namespace orc

using namespace orc;

extern "C" {

int orc_nvar(int ndim, int mhd) {
  Phys p; p.ndim = ndim; p.mhd = mhd; p.gamma = 1.4;
  return p.nvar();
}

// MP5 left-biased interface value from f[0..4] = f_{j-2}..f_{j+2}.
double orc_mp5(const double* f, double eps) { return mp5<double>(f[0], f[1], f[2], f[3], f[4], eps); }

// MP5 and its five partial derivatives (dual numbers, one per input).
double orc_mp5_grad(const double* f, double eps, double* grad) {
  double out = 0.0;
  for (int s = 0; s < 5; ++s) {
    Dual x[5];
    for (int t = 0; t < 5; ++t) x[t] = Dual(f[t], t == s ? 1.0 : 0.0);
    Dual r = mp5<Dual>(x[0], x[1], x[2], x[3], x[4], eps);
    grad[s] = r.d;
    out = r.v;
  }
  return out;
}

// LIM03 left-biased interface value from f[0..2] = f_{j-1}..f_{j+1} on
// cells of width dx.
double orc_lim03(const double* f, double dx) { return lim03<double>(f[0], f[1], f[2], dx); }

// LIM03 and its three partial derivatives.
double orc_lim03_grad(const double* f, double dx, double* grad) {
  double out = 0.0;
  for (int s = 0; s < 3; ++s) {
    Dual x[3];
    for (int t = 0; t < 3; ++t) x[t] = Dual(f[t], t == s ? 1.0 : 0.0);
    Dual r = lim03<Dual>(x[0], x[1], x[2], dx);
    grad[s] = r.d;
    out = r.v;
  }
  return out;
}

// Reconstruction of the following rhs / run / jvp calls: 0 MP5, 1 LIM03.
// Hall parameter eta_h of the following MHD calls (0: ideal MHD).
void orc_set_hall(double eta_h) { g_eta_h = eta_h; }

// Test hook: radius r of LIM03's asymptotic region (default 1).
void orc_set_lim03_radius(double r) { LIM03_RADIUS = r; }

int orc_set_recon(int recon) {
  if (recon != 0 && recon != 1) return ORC_ERR_INVALID;
  g_recon = recon;
  return ORC_OK;
}

// Primitive variables (rho, vx, vy, vz, p, Bx, By, Bz) of one cell.
int orc_prim(int ndim, int mhd, double gamma, const double* u, double* w8) {
  Phys ph; ph.ndim = ndim; ph.mhd = mhd; ph.gamma = gamma;
  Prim<double> w;
  bool ok = cons_to_prim(ph, u, w);
  w8[0] = w.rho; w8[1] = w.v[0]; w8[2] = w.v[1]; w8[3] = w.v[2]; w8[4] = w.p;
  w8[5] = w.B[0]; w8[6] = w.B[1]; w8[7] = w.B[2];
  return ok ? ORC_OK : ORC_ERR_NONPHYSICAL;
}

int orc_flux(int ndim, int mhd, double gamma, int d, const double* u, double* f) {
  Phys ph; ph.ndim = ndim; ph.mhd = mhd; ph.gamma = gamma;
  Prim<double> w;
  bool ok = cons_to_prim(ph, u, w);
  phys_flux(ph, d, u, w, f);
  return ok ? ORC_OK : ORC_ERR_NONPHYSICAL;
}

// GLM flux (reading R8) along d with cleaning speed ch; u and f hold 9 values.
int orc_flux_glm(int ndim, double gamma, int d, double ch, const double* u, double* f) {
  Phys ph; ph.ndim = ndim; ph.mhd = 2; ph.gamma = gamma;
  Prim<double> w;
  bool ok = cons_to_prim(ph, u, w);
  phys_flux(ph, d, u, w, f, ch);
  return ok ? ORC_OK : ORC_ERR_NONPHYSICAL;
}

// MHD flux with the Hall terms (reading R9) for a given current J[3].
int orc_flux_hall(int ndim, double gamma, double eta_h, int d, const double* u, const double* J, double* f) {
  Phys ph; ph.ndim = ndim; ph.mhd = 1; ph.gamma = gamma; ph.eta_h = eta_h;
  Prim<double> w;
  bool ok = cons_to_prim(ph, u, w);
  phys_flux(ph, d, u, w, f, 0.0, J);
  return ok ? ORC_OK : ORC_ERR_NONPHYSICAL;
}

// c_r of the GLM psi decay (reading R8), and a test hook to change it.
double orc_glm_cr(void) { return GLM_CR; }
void orc_set_glm_cr(double cr) { GLM_CR = cr; }

double orc_fast_speed(int ndim, int mhd, double gamma, int d, const double* u) {
  Phys ph; ph.ndim = ndim; ph.mhd = mhd; ph.gamma = gamma;
  Prim<double> w;
  cons_to_prim(ph, u, w);
  return fast_speed(ph, d, w);
}

// Shu-Osher table: alpha, beta are 6x6 row-major (row i = stage i).
int orc_scheme_table(int scheme, double* alpha, double* beta) {
  Scheme S = make_scheme(scheme);
  for (int i = 0; i < 6; ++i)
    for (int k = 0; k < 6; ++k) { alpha[6 * i + k] = S.alpha[i][k]; beta[6 * i + k] = S.beta[i][k]; }
  return S.s;
}

// L(U) on every block.  u: padded input blocks (periodic ghosts are filled
// from neighbours internally; fixed ghosts are read as given).  rhs:
// padded output blocks (ghost entries set to 0).  cmax: out, per direction.
// cmax_in: if non-NULL, c_max to use instead of the maximum over these
// blocks (lets a test evaluate L on a sample of a larger block list).
int orc_rhs(int ndim, int mhd, double gamma, double eps, int nb, const int* n, const double* dx,
            const int* nbr, const double* const* u, double* const* rhs_out, double* cmax,
            const double* cmax_in) {
  Grid G;
  int st = build_grid(G, ndim, mhd, gamma, nb, n, dx, nbr);
  if (st) return st;
  State<double> U, L;
  load_state(G, U, u);
  alloc_state(G, L);
  fill_ghosts(G, U);
  double cm[3];
  st = global_cmax(G, U, cm);
  if (st) return st;
  if (cmax_in)
    for (int d = 0; d < 3; ++d) cm[d] = cmax_in[d];
  st = rhs(G, U, cm, L, eps);
  if (st) return st;
  for (int b = 0; b < nb; ++b) std::memcpy(rhs_out[b], L[b].data(), L[b].size() * sizeof(double));
  for (int d = 0; d < 3; ++d) cmax[d] = cm[d];
  return ORC_OK;
}

// c_max (reading R1) of the interior cells of the given blocks.
int orc_cmax(int ndim, int mhd, double gamma, int nb, const int* n, const double* dx, const int* nbr,
             const double* const* u, double* cmax) {
  Grid G;
  int st = build_grid(G, ndim, mhd, gamma, nb, n, dx, nbr);
  if (st) return st;
  State<double> U;
  load_state(G, U, u);
  double cm[3];
  st = global_cmax(G, U, cm);
  for (int d = 0; d < 3; ++d) cmax[d] = cm[d];
  return st;
}

// Divergence of B at every interior cell by fourth-order central
// differences along each active direction (the monitor of Sect. 4.5.1):
//   div B = sum_d (8 (B_d[i+1] - B_d[i-1]) - (B_d[i+2] - B_d[i-2])) / (12 dx_d),
// halo from the face neighbours (periodic) or the fixed ghost layers.
// out: per block, interior-only layout (one double per cell, x fastest).
int orc_divb(int ndim, int mhd, double gamma, int nb, const int* n, const double* dx, const int* nbr,
             const double* const* u, double* const* out) {
  if (mhd == 0) return ORC_ERR_INVALID;
  Grid G;
  int st = build_grid(G, ndim, mhd, gamma, nb, n, dx, nbr);
  if (st) return st;
  State<double> U;
  load_state(G, U, u);
  fill_ghosts(G, U);
  for (int b = 0; b < nb; ++b) {
    const Geom& q = G.g[b];
    size_t o = 0;
    for (int k = 0; k < q.n[2]; ++k)
      for (int j = 0; j < q.n[1]; ++j)
        for (int i = 0; i < q.n[0]; ++i, ++o) {
          double div = 0.0;
          for (int d = 0; d < ndim; ++d) {
            auto B = [&](int s) {
              int c[3] = {i, j, k};
              c[d] += s;
              return U[b][(5 + d) * q.ncell + q.idx(c[0], c[1], c[2])];
            };
            div = div + (8.0 * (B(1) - B(-1)) - (B(2) - B(-2))) / (12.0 * q.dx[d]);
          }
          out[b][o] = div;
        }
  }
  return ORC_OK;
}

// nsteps SSPRK steps.  dt_fixed <= 0 selects the CFL rule.  u: in/out
// padded blocks (interiors updated; ghosts on output are those of the last
// stage: periodic ones refreshed, fixed ones unchanged).  dts: optional
// array of nsteps used time steps.
int orc_run(int ndim, int mhd, double gamma, double eps, int nb, const int* n, const double* dx,
            const int* nbr, int scheme, double cfl, double dt_fixed, int nsteps,
            double* const* u, double* dts) {
  Grid G;
  int st = build_grid(G, ndim, mhd, gamma, nb, n, dx, nbr);
  if (st) return st;
  if (scheme < 0 || scheme > 2) return ORC_ERR_INVALID;
  Scheme S = make_scheme(scheme);
  State<double> U;
  load_state(G, U, u);
  for (int it = 0; it < nsteps; ++it) {
    double dtu = 0.0;
    st = ssprk_step(G, S, U, cfl, dt_fixed > 0.0 ? dt_fixed : -1.0, eps, &dtu);
    if (st) return st;
    if (dts) dts[it] = dtu;
  }
  fill_ghosts(G, U);
  for (int b = 0; b < nb; ++b) std::memcpy(u[b], U[b].data(), U[b].size() * sizeof(double));
  return ORC_OK;
}

// Jacobian-vector product of the map U_0 -> U_N (N = nsteps, fixed dt):
// u in/out (value), du in/out (tangent).  Forward-mode dual numbers through
// every stage, including the global c_max (derivative of the maximising
// cell).
int orc_run_jvp(int ndim, int mhd, double gamma, double eps, int nb, const int* n,
                const double* dx, const int* nbr, int scheme, double dt, int nsteps,
                double* const* u, double* const* du) {
  Grid G;
  int st = build_grid(G, ndim, mhd, gamma, nb, n, dx, nbr);
  if (st) return st;
  if (scheme < 0 || scheme > 2 || !(dt > 0.0)) return ORC_ERR_INVALID;
  Scheme S = make_scheme(scheme);
  State<Dual> U;
  alloc_state(G, U);
  for (int b = 0; b < nb; ++b)
    for (size_t o = 0; o < U[b].size(); ++o) U[b][o] = Dual(u[b][o], du[b][o]);
  for (int it = 0; it < nsteps; ++it) {
    st = ssprk_step(G, S, U, 0.0, dt, eps, nullptr);
    if (st) return st;
  }
  fill_ghosts(G, U);
  for (int b = 0; b < nb; ++b)
    for (size_t o = 0; o < U[b].size(); ++o) { u[b][o] = U[b][o].v; du[b][o] = U[b][o].d; }
  return ORC_OK;
}

// Reverse mode (vector-Jacobian product) of nsteps steps at fixed dt from
// U_0 = u (padded blocks, read only): lam (padded blocks) holds dJ/dU_N on
// entry (ghost entries ignored) and on return dJ/dU_0 in the interiors, the
// adjoint of the boundary data in the face ghosts of fixed faces (nbr < 0),
// and 0 in every other ghost entry.  All stage states of every step are
// recomputed from stored step states.  Ideal hydro and MHD, MP5 or LIM03;
// GLM, Hall MHD and passive blocks are refused.
int orc_run_vjp(int ndim, int mhd, double gamma, double eps, int nb, const int* n, const double* dx,
                const int* nbr, int scheme, double dt, int nsteps, double* const* u, double* const* lam) {
  Grid G;
  int st = build_grid(G, ndim, mhd, gamma, nb, n, dx, nbr);
  if (st) return st;
  if (scheme < 0 || scheme > 2 || !(dt > 0.0) || nsteps < 0 || mhd == 2 || G.ph.eta_h != 0.0 ||
      !G.active.empty())
    return ORC_ERR_INVALID;
  Scheme S = make_scheme(scheme);
  std::vector<State<double>> Ustep(nsteps);
  State<double> U;
  load_state(G, U, u);
  for (int it = 0; it < nsteps; ++it) {
    Ustep[it] = U;
    st = ssprk_step(G, S, U, 0.0, dt, eps, nullptr);
    if (st) return st;
  }
  State<double> L, gadj;
  alloc_state(G, L);
  alloc_state(G, gadj);
  for (int b = 0; b < nb; ++b) {
    const Geom& q = G.g[b];
    for (int k = 0; k < q.n[2]; ++k)
      for (int j = 0; j < q.n[1]; ++j)
        for (int i = 0; i < q.n[0]; ++i)
          for (int v = 0; v < G.ph.nvar(); ++v) {
            const size_t o = v * q.ncell + q.idx(i, j, k);
            L[b][o] = lam[b][o];
          }
  }
  for (int it = nsteps - 1; it >= 0; --it) {
    st = ssprk_step_vjp(G, S, Ustep[it], dt, eps, L, gadj);
    if (st) return st;
    Ustep[it].clear();
  }
  for (int b = 0; b < nb; ++b)
    for (size_t o = 0; o < L[b].size(); ++o) lam[b][o] = L[b][o] + gadj[b][o];
  return ORC_OK;
}

// Operation counts of one step of `scheme` (CFL 0.4) on the given blocks,
// single-threaded: per category (0 other, 1 primitive recovery + flux +
// split of one cell along one direction, 2 reconstructions (two per
// interface and variable, with the sum of the pair), 3 conservative
// difference (per cell, variable and direction), 4 c_max (per cell, every
// direction), 5 stage combination (per cell and stage)) the arithmetic
// operations nops, the comparisons and selections ncmp, and the units.
// median_form != 0 evaluates MP5 without its early exit.
int orc_count_ops(int ndim, int mhd, double gamma, double eps, int nb, const int* n, const double* dx,
                  const int* nbr, const double* const* u, int scheme, int median_form, uint64_t* nops,
                  uint64_t* ncmp, uint64_t* units) {
  Grid G;
  int st = build_grid(G, ndim, mhd, gamma, nb, n, dx, nbr);
  if (st) return st;
  if (scheme < 0 || scheme > 2) return ORC_ERR_INVALID;
  Scheme S = make_scheme(scheme);
  State<Counted> U;
  alloc_state(G, U);
  for (int b = 0; b < nb; ++b)
    for (size_t o = 0; o < U[b].size(); ++o) U[b][o] = Counted(u[b][o]);
#ifdef _OPENMP
  const int threads = omp_get_max_threads();
  omp_set_num_threads(1);
#endif
  for (int c = 0; c < NCAT; ++c) g_nops[c] = g_ncmp[c] = g_units[c] = 0;
  g_mp5_median = median_form != 0;
  g_count_on = true;
  g_cat = CAT_OTHER;
  st = ssprk_step(G, S, U, 0.4, -1.0, eps, nullptr);
  g_count_on = false;
  g_mp5_median = false;
#ifdef _OPENMP
  omp_set_num_threads(threads);
#endif
  for (int c = 0; c < NCAT; ++c) {
    nops[c] = g_nops[c];
    ncmp[c] = g_ncmp[c];
    units[c] = g_units[c];
  }
  return st;
}

// Test hook: MP5 without its early exit (the median form) in later calls.
void orc_set_mp5_median(int on) { g_mp5_median = on != 0; }

// Branch fingerprint: orc_branch_hash_begin() enables collection (and
// forces one thread), orc_branch_hash_end() returns the fingerprint.
void orc_branch_hash_begin(void) {
  g_hash_on = true;
  g_hash = 1469598103934665603ull;
#ifdef _OPENMP
  omp_set_num_threads(1);
#endif
}

uint64_t orc_branch_hash_end(void) {
  g_hash_on = false;
  return g_hash;
}

// Active flags (one byte per block, nonzero = active) used by the grids of
// every later call with the same number of blocks; n = 0 or flags = NULL
// makes every block active again.
void orc_set_active(const unsigned char* flags, int n) {
  g_active.clear();
  if (flags && n > 0) g_active.assign(flags, flags + n);
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
