// Device arithmetic shared by the forward stage kernel and the adjoint:
// state addressing, primitive recovery, physical flux, fast and whistler
// speeds, MP5 and LIM03, tile geometry and the XCD-aware tile schedule.
// Sharing one definition makes the adjoint's recompute of the forward pass
// bitwise identical to the forward pass (no automatic FMA contraction; every
// fused multiply-add is explicit).
#pragma once
#include "amrvac_internal.h"

#include <type_traits>
#include <utility>

namespace amrvac {

// Variables: hydro (rho, m_1..m_NDIM, E); MHD (rho, m_x, m_y, m_z, E, B_x,
// B_y, B_z); GLM as MHD, then psi.
template <int NDIM, bool MHD, bool GLM = false>
struct Eq {
  static_assert(MHD || !GLM, "GLM extends MHD");
  static constexpr int NV = GLM ? 9 : MHD ? 8 : 2 + NDIM;
  static constexpr int NC = MHD ? 3 : NDIM;
  static constexpr int IE = 1 + NC;
};

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// ---------------------------------------------------------------------------
// Addressing of state buffers.
// ---------------------------------------------------------------------------
// A wave-uniform int the compiler must treat as unknown at this point: the
// stage update's buffer addresses derived from it are then rebuilt per tile
// (a few scalar operations) instead of being hoisted out of the tile loop and
// held, or spilled, across it.  The empty asm emits no instruction.
__device__ __forceinline__ int opaque_uniform(int x) {
  asm volatile("" : "+s"(x));
  return x;
}

// The same value, hidden from common-subexpression elimination (no
// instruction): a recomputation from it is not merged with an earlier one,
// so the earlier results need not stay live in registers until then.
__device__ __forceinline__ double opaque_value(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Pointers into global memory (address space 1).  Block states and scratch
// slots are reached through pointers read from the block table, which the
// compiler would otherwise treat as generic: generic accesses compile to
// flat instructions, whose completion the LDS counter waits for as well, so
// every LDS wait would also wait for the global loads in flight.
using gptr = __attribute__((address_space(1))) const double*;
using gptr_w = __attribute__((address_space(1))) double*;

__device__ __forceinline__ gptr cell_addr(const StateTable& st, const BlockDev& B, int buf, int i, int j, int k,
                                          long long& vstride) {
  if (buf == 0) {
    vstride = (long long)B.P[0] * B.P[1] * B.P[2];
    return (gptr)(B.u + (((long long)(k + B.g[2]) * B.P[1] + (j + B.g[1])) * B.P[0] + (i + B.g[0])));
  }
  vstride = B.cells;
  return (gptr)(st.scr + (long long)(buf - 1) * st.slot_stride + B.off + (((long long)k * B.n[1] + j) * B.n[0] + i));
}

__device__ __forceinline__ gptr_w cell_addr_w(const StateTable& st, const BlockDev& B, int buf, int i, int j, int k,
                                              long long& vstride) {
  return (gptr_w)cell_addr(st, B, buf, i, j, k, vstride);
}

// Load all NV variables of cell (i,j,k) of block blk, where only coordinate
// D may lie outside [0, n_D): then the value comes from the face neighbour's
// interior (same buffer), or from this block's fixed ghost layer (buffer 0).
template <int NV, int D>
__device__ __forceinline__ void load_cell(const StateTable& st, int blk, int buf, int i, int j, int k,
                                          double* u) {
  const BlockDev* B = &st.blocks[blk];
  int c[3] = {i, j, k};
  int bf = buf;
  if (c[D] < 0) {
    int nb = B->nbr[2 * D];
    if (nb >= 0) {
      B = &st.blocks[nb];
      c[D] += B->n[D];
    } else {
      bf = 0;
    }
  } else if (c[D] >= B->n[D]) {
    int nb = B->nbr[2 * D + 1];
    if (nb >= 0) {
      c[D] -= B->n[D];
      B = &st.blocks[nb];
    } else {
      bf = 0;
    }
  }
  long long vs;
  gptr p = cell_addr(st, *B, bf, c[0], c[1], c[2], vs);
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = p[v * vs];
}

// As load_cell, for the variables V0 .. V0+VN-1 only.
template <int V0, int VN, int D>
__device__ __forceinline__ void load_cell_vars(const StateTable& st, int blk, int buf, int i, int j, int k,
                                               double* u) {
  const BlockDev* B = &st.blocks[blk];
  int c[3] = {i, j, k};
  int bf = buf;
  if (c[D] < 0) {
    int nb = B->nbr[2 * D];
    if (nb >= 0) {
      B = &st.blocks[nb];
      c[D] += B->n[D];
    } else {
      bf = 0;
    }
  } else if (c[D] >= B->n[D]) {
    int nb = B->nbr[2 * D + 1];
    if (nb >= 0) {
      c[D] -= B->n[D];
      B = &st.blocks[nb];
    } else {
      bf = 0;
    }
  }
  long long vs;
  gptr p = cell_addr(st, *B, bf, c[0], c[1], c[2], vs);
#pragma unroll
  for (int v = 0; v < VN; ++v) u[v] = p[(V0 + v) * vs];
}

// Value of plane v of a per-cell array (interior layout, block at coff, plane
// stride `plane`) at cell (i,j,k) of block blk, where only coordinate D may
// lie outside the block: then the face neighbour's cell (its face must
// exist).
template <int D>
__device__ __forceinline__ double load_plane(const StateTable& st, const double* a, long long plane, int v, int blk,
                                             int i, int j, int k) {
  const BlockDev* B = &st.blocks[blk];
  int c[3] = {i, j, k};
  if (c[D] < 0) {
    B = &st.blocks[B->nbr[2 * D]];
    c[D] += B->n[D];
  } else if (c[D] >= B->n[D]) {
    c[D] -= B->n[D];
    B = &st.blocks[B->nbr[2 * D + 1]];
  }
  return ((gptr)a)[v * plane + B->coff + ((long long)c[2] * B->n[1] + c[1]) * B->n[0] + c[0]];
}

// ---------------------------------------------------------------------------
// Physics: primitive recovery, flux along D, fast speed.
// ---------------------------------------------------------------------------
struct PrimD {
  double rho, ri, v[3], p, B[3], b2;
};

template <int NDIM, bool MHD>
__device__ __forceinline__ bool prim(const double* u, double gamma, PrimD& w) {
  using E = Eq<NDIM, MHD>;
  w.rho = u[0];
  w.ri = 1.0 / w.rho;
  double mv = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    w.v[k] = (k < E::NC) ? u[1 + k] * w.ri : 0.0;
    w.B[k] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < E::NC; ++k) mv = fma(u[1 + k], w.v[k], mv);
  double eint = fma(-0.5, mv, u[E::IE]);
  w.b2 = 0.0;
  if constexpr (MHD) {
#pragma unroll
    for (int k = 0; k < 3; ++k) w.B[k] = u[5 + k];
    w.b2 = fma(w.B[2], w.B[2], fma(w.B[1], w.B[1], w.B[0] * w.B[0]));
    eint = fma(-0.5, w.b2, eint);
  }
  w.p = (gamma - 1.0) * eint;
  return (w.rho > 0.0) && (w.p > 0.0) && (w.p < __builtin_huge_val()) &&
         (w.rho < __builtin_huge_val());
}

// Physical flux along D (Sect. 3 eqs. masscons, momentum, total; Sect. 4.1
// eq. b1eq and Sect. 4.3 eqs. momentummhd, fractional with B0 = 0).
template <int NDIM, bool MHD, int D>
__device__ __forceinline__ void phys_flux(const double* u, const PrimD& w, double* F) {
  using E = Eq<NDIM, MHD>;
  const double vd = w.v[D];
  F[0] = u[1 + D];
  if constexpr (!MHD) {
#pragma unroll
    for (int k = 0; k < E::NC; ++k) F[1 + k] = u[1 + k] * vd;
    F[1 + D] += w.p;
    F[E::IE] = vd * (u[E::IE] + w.p);
  } else {
    const double ptot = fma(0.5, w.b2, w.p);
    const double Bd = w.B[D];
    const double bv = fma(w.B[2], w.v[2], fma(w.B[1], w.v[1], w.B[0] * w.v[0]));
#pragma unroll
    for (int k = 0; k < 3; ++k) F[1 + k] = fma(u[1 + k], vd, -(Bd * w.B[k]));
    F[1 + D] += ptot;
    F[4] = fma(vd, u[4] + ptot, -(Bd * bv));
#pragma unroll
    for (int k = 0; k < 3; ++k) F[5 + k] = (k == D) ? 0.0 : fma(vd, w.B[k], -(Bd * w.v[k]));
  }
}

// Hall MHD: the fast whistler speed eta_h |B| k_max / rho at k_max = pi
// max_d 1/dx_d of the block (Sect. 4.4).
__device__ __forceinline__ double whistler_speed(const PrimD& w, double eta_h, double kmax) {
  const double babs = sqrt(w.B[0] * w.B[0] + w.B[1] * w.B[1] + w.B[2] * w.B[2]);
  return eta_h * babs / w.rho * kmax;
}

// Fast magnetosonic speed along d (sound speed for hydro).
template <bool MHD>
__device__ __forceinline__ double fast_speed(const PrimD& w, int d, double gamma) {
  const double a2 = gamma * w.p * w.ri;
  if constexpr (!MHD) {
    return sqrt(a2);
  } else {
    const double b2 = w.b2 * w.ri;
    const double bd2 = w.B[d] * w.B[d] * w.ri;
    const double s = a2 + b2;
    double disc = fma(s, s, -4.0 * a2 * bd2);
    disc = disc < 0.0 ? 0.0 : disc;
    return sqrt(0.5 * (s + sqrt(disc)));
  }
}

// ---------------------------------------------------------------------------
// MP5 (Suresh & Huynh 1997), alpha = 4, eps = 0, median form.
// ---------------------------------------------------------------------------
// minmod of four arguments (the one of smallest magnitude when all have
// the same sign, else zero), as a clamp of zero into [min, max]: the result
// is one of the arguments exactly, or zero.
__device__ __forceinline__ double minmod4(double w, double x, double y, double z) {
  const double lo = fmin(fmin(w, x), fmin(y, z));
  const double hi = fmax(fmax(w, x), fmax(y, z));
  return fmax(lo, fmin(hi, 0.0));
}

// Curvature limiter of the cell pair (j, j+1) from their curvatures x = d_j
// and y = d_{j+1}: d^M4_{j+1/2}.  Both limiters of a reconstruction use it
// with the lower cell first, so neighbouring interfaces of a pencil share
// one evaluation.
__device__ __forceinline__ double m4pair(double x, double y) {
  return minmod4(fma(4.0, x, -y), fma(4.0, y, -x), x, y);
}

// Bounds and clamp of MP5 from the stencil centre c, its right neighbour
// d, the fifth-order value fL, c - b and the two curvature limiters.
struct Mp5Parts {
  double fUL, fMD, fLC, fmn, fmx;
  double amn, amx;   // the (c, d, fMD) halves of fmn and fmx
};
__device__ __forceinline__ double mp5_tail(double c, double d, double fL, double cb, double m4p, double m4m,
                                           Mp5Parts& q) {
  q.fUL = fma(4.0, cb, c);
  q.fMD = fma(-0.5, m4p, 0.5 * (c + d));
  q.fLC = fma(4.0 / 3.0, m4m, fma(0.5, cb, c));
  q.amn = fmin(fmin(c, d), q.fMD);
  q.amx = fmax(fmax(c, d), q.fMD);
  q.fmn = fmax(q.amn, fmin(fmin(c, q.fUL), q.fLC));
  q.fmx = fmin(q.amx, fmax(fmax(c, q.fUL), q.fLC));
  return fmin(fmax(fL, q.fmn), q.fmx);
}

// Linear pieces of MP5.  With eps = 0, mp5 is continuous and piecewise
// linear in its five inputs; mp5_piece names the piece it evaluates (the
// adjoint multiplies by that piece's constant weights):
//   0 fL;  1 c;  2 d;  3 fUL;  4 + k fMD and 9 + k fLC, where k (0..4) is
//   the argument the curvature minmod returned, k = 0 for zero, with the
//   arguments ordered (4d_j - d_{j+1}, 4d_{j+1} - d_j, d_j, d_{j+1}) for fMD
//   at j+1/2 and (4d_j - d_{j-1}, 4d_{j-1} - d_j, d_j, d_{j-1}) for fLC at
//   j-1/2.  The piece is fL when fmin <= fL <= fmax; else the candidate that
//   realised the bound r the value was clamped to (fmin when fL < fmin, fmax
//   when fL > fmax).  The bound is the max (min) of two chains, (c, d, fMD)
//   and (c, fUL, fLC), and the first chain wins ties, so r comes from the
//   second chain exactly when it differs from the first chain's value; in
//   that chain the piece is the first candidate equal to r, which is the
//   earlier-wins tie rule of the min/max chains.
__device__ __forceinline__ int mp5_piece(double c, double d, double fL, const Mp5Parts& q, int kp, int km) {
  const bool lo = fL < q.fmn, hi = fL > q.fmx;
  const double r = lo ? q.fmn : q.fmx;
  const bool second = r != (lo ? q.amn : q.amx);
  const int k = c == r ? 1 : second ? (q.fUL == r ? 3 : 9 + km) : (d == r ? 2 : 4 + kp);
  return (lo || hi) ? k : 0;
}

// MP5 (Suresh & Huynh 1997, alpha = 4, eps = 0, median form) of RUN
// consecutive interfaces of a pencil: interface kk reconstructs from the
// stencil f[kk .. kk+4] (f_{j-2} .. f_{j+2}).  Curvatures and curvature
// limiters are evaluated once and shared by the interfaces that use them;
// every value is bitwise that of RUN separate evaluations.  With CODES the
// linear piece of every interface is returned as well.
template <int RUN, bool CODES>
__device__ __forceinline__ void mp5_run(const double* f, double* out, int* code) {
  double dc[RUN + 2];   // curvature at stencil position j + 1
#pragma unroll
  for (int j = 0; j < RUN + 2; ++j) dc[j] = fma(-2.0, f[j + 1], f[j]) + f[j + 2];
  double m4[RUN + 1];   // limiter of the pair (j + 1, j + 2)
#pragma unroll
  for (int j = 0; j < RUN + 1; ++j) m4[j] = m4pair(dc[j], dc[j + 1]);
  auto fifth = [&](int kk) {
    return fma(2.0, f[kk], fma(-13.0, f[kk + 1], fma(47.0, f[kk + 2], fma(27.0, f[kk + 3], -3.0 * f[kk + 4])))) *
           (1.0 / 60.0);
  };
  bool clamped = false;
#pragma unroll
  for (int kk = 0; kk < RUN; ++kk) {
    const double fL = fifth(kk);
    Mp5Parts q;
    out[kk] = mp5_tail(f[kk + 2], f[kk + 3], fL, f[kk + 2] - f[kk + 1], m4[kk + 1], m4[kk], q);
    if constexpr (CODES) clamped = clamped || out[kk] != fL;   // fL < fmin or fL > fmax
  }
  if constexpr (CODES) {
    // every piece is fL (code 0) unless the value was clamped; a wave in
    // which no lane clamped any interface of its run skips the search
    if (__ballot(clamped) == 0) {
#pragma unroll
      for (int kk = 0; kk < RUN; ++kk) code[kk] = 0;
      return;
    }
    // Recomputed from the stencil values (passed through opaque_value, so
    // that nothing of the first pass stays live for this rare path): the
    // same operations on the same inputs give the same curvatures, limiters,
    // fifth-order values and bounds.
    double g[RUN + 4];
#pragma unroll
    for (int j = 0; j < RUN + 4; ++j) g[j] = opaque_value(f[j]);
    double gc[RUN + 2];
#pragma unroll
    for (int j = 0; j < RUN + 2; ++j) gc[j] = fma(-2.0, g[j + 1], g[j]) + g[j + 2];
    // the argument each pair limiter returned, in the two orders its
    // interfaces number them: (4x - y, 4y - x, x, y) where it is the limiter
    // at j+1/2 (fMD of interface kk = pair - 1), and (4y - x, 4x - y, y, x)
    // where it is the limiter at j-1/2 (fLC of interface kk = pair)
    double gm[RUN + 1];
    int kpp[RUN + 1], kmp[RUN + 1];
#pragma unroll
    for (int j = 0; j < RUN + 1; ++j) {
      const double x = gc[j], y = gc[j + 1];
      const double m = m4pair(x, y);
      gm[j] = m;
      const bool z = m == 0.0, e1 = fma(4.0, x, -y) == m, e2 = fma(4.0, y, -x) == m, e3 = x == m, e4 = y == m;
      kpp[j] = z ? 0 : e1 ? 1 : e2 ? 2 : e3 ? 3 : 4;
      kmp[j] = z ? 0 : e2 ? 1 : e1 ? 2 : e4 ? 3 : 4;
    }
#pragma unroll
    for (int kk = 0; kk < RUN; ++kk) {
      const double fL =
          fma(2.0, g[kk], fma(-13.0, g[kk + 1], fma(47.0, g[kk + 2], fma(27.0, g[kk + 3], -3.0 * g[kk + 4])))) *
          (1.0 / 60.0);
      Mp5Parts q;
      (void)mp5_tail(g[kk + 2], g[kk + 3], fL, g[kk + 2] - g[kk + 1], gm[kk + 1], gm[kk], q);
      code[kk] = mp5_piece(g[kk + 2], g[kk + 3], fL, q, kpp[kk + 1], kmp[kk]);
    }
  }
}

__device__ __forceinline__ double mp5(double a, double b, double c, double d, double e) {
  const double f[5] = {a, b, c, d, e};
  double r;
  mp5_run<1, false>(f, &r, nullptr);
  return r;
}

// ---------------------------------------------------------------------------
// LIM03 (Cada & Torrilhon 2009): compact third-order reconstruction with the
// asymptotic-region switch.
// ---------------------------------------------------------------------------
// Radius r of the asymptotic region, in units of the data per cell width.
constexpr double LIM03_RADIUS = 1.0;

// Interface value at j+1/2 from a = f_{j-1}, b = f_j, c = f_{j+1}; kr =
// 1 / (r dx)^2 for the cell width dx along the pencil.  With dm = b - a and
// dp = c - b the value is b + H/2, where
//   H = (2 dp + dm)/3                      if (dm^2 + dp^2) kr <= 1,
//   H = phi(dm/dp) dp                      otherwise,
//   phi(t) = max(0, min(phi3, max(-t/2, min(2t, phi3, 1.6)))), phi3 = (2+t)/3.
// The limited branch is evaluated without a division: with s = sign(dp)
// and p3 = (2 dp + dm)/3,
//   phi(dm/dp) dp = s max(0, min(s p3, max(-s dm/2, min(2 s dm, s p3, 1.6 |dp|)))),
// which is 0 for dp = 0 (the limit of both one-sided branches).
// The function is piecewise linear in (a, b, c); with CODES the piece is
// returned for the adjoint: 0 H = 0; 1 the third-order formula (either
// branch); 2 -theta/2; 3 2 theta; 4 the 1.6 cap.
template <bool CODES>
__device__ __forceinline__ double lim03_eval(double a, double b, double c, double kr, int& code) {
  const double dm = b - a, dp = c - b;
  const double p3 = fma(2.0, dp, dm) * (1.0 / 3.0);
  const double eta = fma(dm, dm, dp * dp) * kr;
  const double s = dp > 0.0 ? 1.0 : (dp < 0.0 ? -1.0 : 0.0);
  const double sp3 = s * p3, sdm = s * dm, adp = s * dp;
  const double q = -0.5 * sdm, t = 2.0 * sdm, g = 1.6 * adp;
  const double lo = fmin(sp3, fmax(q, fmin(fmin(t, sp3), g)));
  const bool asym = eta <= 1.0;
  const double h = asym ? p3 : s * fmax(0.0, lo);
  if constexpr (CODES) {
    code = asym ? 1 : (!(lo > 0.0) || s == 0.0) ? 0 : lo == sp3 ? 1 : lo == q ? 2 : lo == t ? 3 : 4;
  }
  return fma(0.5, h, b);
}

__device__ __forceinline__ double lim03(double a, double b, double c, double kr) {
  int unused;
  return lim03_eval<false>(a, b, c, kr, unused);
}

// ---------------------------------------------------------------------------
// Tile geometry helpers (compile time).
// ---------------------------------------------------------------------------
template <int TX, int TY, int TZ, int HG = NG>
struct TileShape {
  static constexpr int T(int d) { return d == 0 ? TX : d == 1 ? TY : TZ; }
  static constexpr int TC = TX * TY * TZ;
  // extended box along D (halo of HG cells on both sides: 3 for MP5, 2 for
  // LIM03)
  static constexpr int E(int D, int d) { return T(d) + (d == D ? 2 * HG : 0); }
  static constexpr int NEXT(int D) { return E(D, 0) * E(D, 1) * E(D, 2); }
  static constexpr int SD(int D) { return D == 0 ? 1 : D == 1 ? E(D, 0) : E(D, 0) * E(D, 1); }
  // interface box along D
  static constexpr int I(int D, int d) { return T(d) + (d == D ? 1 : 0); }
  static constexpr int NIFC(int D) { return I(D, 0) * I(D, 1) * I(D, 2); }
  static constexpr int SI(int D) { return D == 0 ? 1 : D == 1 ? I(D, 0) : I(D, 0) * I(D, 1); }
};

template <int A, int B>
struct cmax_i { static constexpr int v = A > B ? A : B; };

// XCD-aware persistent tile schedule.  Work-groups of a launch are
// dispatched round-robin over the 8 XCDs (work-group w on XCD w % 8), each
// XCD with its own L2.  The tile list (Morton-ordered, so contiguous ranges
// are compact in space) is cut into 8 contiguous chunks and chunk x is
// processed only by the work-groups of XCD x, so tiles whose halos overlap
// mostly share one L2.  Every tile is visited exactly once; with fewer than
// 8 work-groups the schedule is the plain grid stride.
struct TileSchedule {
  int t, end, step;
  __device__ __forceinline__ TileSchedule(int ntiles) {
    const int G = (int)gridDim.x, w = (int)blockIdx.x;
    if (G < 8) {
      t = w;
      end = ntiles;
      step = G;
    } else {
      const int x = w & 7, r = w >> 3;
      const int gx = (G - x + 7) >> 3;   // work-groups on XCD x
      t = (int)((long long)ntiles * x / 8) + r;
      end = (int)((long long)ntiles * (x + 1) / 8);
      step = gx;
    }
  }
};

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = fmax(x, __shfl_xor(x, m, 64));
  return x;
}

// Sum over the 64 lanes of a wave in a fixed butterfly order (deterministic).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = x + __shfl_xor(x, m, 64);
  return x;
}

}  // namespace amrvac
