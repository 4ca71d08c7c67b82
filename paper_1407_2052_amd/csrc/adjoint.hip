// Reverse mode of the FD-MP5 / global-LF right-hand side (Porth et al. 2014,
// Sects. 2.1-2.2) on gfx950, used by the adjoint of the SSPRK time
// integration (Sect. 2.3).
//
// k_vjp computes lam += scale * J_L(U)^T mu for the local dependence of L
// on U (everything but the global c_max), as a gather per cell so that no
// atomics are needed and the result is deterministic.  Per tile, direction D
// and variable group:
//   A) F+ and F- of the tile extended by 5 cells along D (recomputed with the
//      forward's own device functions, so bitwise equal to the forward), and
//      mu on the tile extended by 3 cells, into LDS;
//   B) for every interface i+1/2 with i in [o-3, o+T+2): the interface
//      adjoint lamFhat = (mu_{i+1} - mu_i) / dx and the linear piece of MP5
//      taken at the F+ and F- stencils.  MP5 with eps = 0 is continuous and
//      piecewise linear, so each piece is one of 14 constant weight vectors
//      and is stored as a one-byte code;
//   C) for every owned cell j: lamF+_j = sum_{i=j-2..j+2} lamFhat_i w+_i,
//      lamF-_j = sum_{i=j-3..j+1} lamFhat_i w-_i (fixed order), then the
//      split adjoint (lamF = (lamF+ + lamF-)/2, c (lamF+ - lamF-)/2) and the
//      transpose of the flux Jacobian (hand-written reverse of the primitive
//      recovery and flux).
// The c_max term sum_j U_j (lamF+_j - lamF-_j)/2 is summed per tile; a
// second kernel adds its product with d(|v_d| + c_f,d)/dU at the maximising
// cell (lowest block, then lowest cell index, on ties).
#include "device_math.h"

namespace amrvac {

// Weights of the five MP5 inputs (f_{j-2} .. f_{j+2}) for each linear piece:
// 0 fL; 1 c; 2 d; 3 fUL; 4+k fMD with the k-th argument of the curvature
// minmod at j+1/2 (k = 0: zero); 9+k fLC with the k-th argument at j-1/2.
__constant__ double c_mp5w[14][5] = {
    {2.0 / 60.0, -13.0 / 60.0, 47.0 / 60.0, 27.0 / 60.0, -3.0 / 60.0},
    {0.0, 0.0, 1.0, 0.0, 0.0},
    {0.0, 0.0, 0.0, 1.0, 0.0},
    {0.0, -4.0, 5.0, 0.0, 0.0},
    {0.0, 0.0, 0.5, 0.5, 0.0},
    {0.0, -2.0, 5.0, -2.5, 0.5},
    {0.0, 0.5, -2.5, 5.0, -2.0},
    {0.0, -0.5, 1.5, 0.0, 0.0},
    {0.0, 0.0, 0.0, 1.5, -0.5},
    {0.0, -0.5, 1.5, 0.0, 0.0},
    {-4.0 / 3.0, 7.5, -10.5, 16.0 / 3.0, 0.0},
    {16.0 / 3.0, -12.5, 9.5, -4.0 / 3.0, 0.0},
    {0.0, 5.0 / 6.0, -7.0 / 6.0, 4.0 / 3.0, 0.0},
    {4.0 / 3.0, -19.0 / 6.0, 17.0 / 6.0, 0.0, 0.0},
};

// Argument (1..4) that minmod4 returns, 0 when it returns zero; ties go to
// the earlier argument.
__device__ __forceinline__ int minmod4_pick(double w, double x, double y, double z) {
  if (w > 0.0 && x > 0.0 && y > 0.0 && z > 0.0) {
    int k = 1;
    double m = w;
    if (x < m) { m = x; k = 2; }
    if (y < m) { m = y; k = 3; }
    if (z < m) { k = 4; }
    return k;
  }
  if (w < 0.0 && x < 0.0 && y < 0.0 && z < 0.0) {
    int k = 1;
    double m = w;
    if (x > m) { m = x; k = 2; }
    if (y > m) { m = y; k = 3; }
    if (z > m) { k = 4; }
    return k;
  }
  return 0;
}

// Linear piece of mp5(a, b, c, d, e) (same arithmetic as the forward): the
// forward returns clamp(fL, fmin, fmax); ties go to fL, and within min/max
// chains to the earlier candidate.
__device__ __forceinline__ int mp5_code(double a, double b, double c, double d, double e) {
  const double fL = fma(2.0, a, fma(-13.0, b, fma(47.0, c, fma(27.0, d, -3.0 * e)))) * (1.0 / 60.0);
  const double cb = c - b;
  const double dm = fma(-2.0, b, a) + c;
  const double d0 = fma(-2.0, c, b) + d;
  const double dp = fma(-2.0, d, c) + e;
  const double w1p = fma(4.0, d0, -dp), w2p = fma(4.0, dp, -d0);
  const double w1m = fma(4.0, d0, -dm), w2m = fma(4.0, dm, -d0);
  const double m4p = minmod4(w1p, w2p, d0, dp);
  const double m4m = minmod4(w1m, w2m, d0, dm);
  const int kp = minmod4_pick(w1p, w2p, d0, dp);
  const int km = minmod4_pick(w1m, w2m, d0, dm);
  const double fUL = fma(4.0, cb, c);
  const double fMD = fma(-0.5, m4p, 0.5 * (c + d));
  const double fLC = fma(4.0 / 3.0, m4m, fma(0.5, cb, c));
  double v1 = c, v2 = c, u1 = c, u2 = c;
  int k1 = 1, k2 = 1, j1 = 1, j2 = 1;
  if (d < v1) { v1 = d; k1 = 2; }
  if (fMD < v1) { v1 = fMD; k1 = 4 + kp; }
  if (fUL < v2) { v2 = fUL; k2 = 3; }
  if (fLC < v2) { v2 = fLC; k2 = 9 + km; }
  if (d > u1) { u1 = d; j1 = 2; }
  if (fMD > u1) { u1 = fMD; j1 = 4 + kp; }
  if (fUL > u2) { u2 = fUL; j2 = 3; }
  if (fLC > u2) { u2 = fLC; j2 = 9 + km; }
  double lo = v1, hi = u1;
  int klo = k1, khi = j1;
  if (v2 > lo) { lo = v2; klo = k2; }
  if (u2 < hi) { hi = u2; khi = j2; }
  if (fL < lo) return klo;
  if (fL > hi) return khi;
  return 0;
}

// Reverse of the primitive recovery: adjoints of the primitives (lv, lp,
// lri = d/d(1/rho), lB = d/dB used directly) accumulated into lu.
template <int NDIM, bool MHD>
__device__ __forceinline__ void prim_vjp(const double* u, const PrimD& w, double gamma, const double* lv, double lp,
                                         double lri, const double* lB, double* lu) {
  using E = Eq<NDIM, MHD>;
  const double le = (gamma - 1.0) * lp;   // adjoint of the internal energy
  lu[E::IE] += le;
  double lvv[3] = {lv[0], lv[1], lv[2]};
#pragma unroll
  for (int k = 0; k < E::NC; ++k) {
    lu[1 + k] += -0.5 * le * w.v[k];
    lvv[k] += -0.5 * le * u[1 + k];
  }
  if constexpr (MHD) {
#pragma unroll
    for (int k = 0; k < 3; ++k) lu[5 + k] += lB[k] - le * w.B[k];
  }
  double lr = lri;
#pragma unroll
  for (int k = 0; k < E::NC; ++k) {
    lu[1 + k] += lvv[k] * w.ri;
    lr += lvv[k] * u[1 + k];
  }
  lu[0] += -lr * w.ri * w.ri;
}

// lu += (dF_D/dU)^T lamF (reverse of phys_flux).
template <int NDIM, bool MHD, int D>
__device__ __forceinline__ void flux_vjp(const double* u, const PrimD& w, double gamma, const double* lF,
                                         double* lu) {
  using E = Eq<NDIM, MHD>;
  const double vd = w.v[D];
  double lv[3] = {0.0, 0.0, 0.0}, lB[3] = {0.0, 0.0, 0.0};
  double lp = 0.0;
  lu[1 + D] += lF[0];
  if constexpr (!MHD) {
#pragma unroll
    for (int k = 0; k < E::NC; ++k) {
      lu[1 + k] += lF[1 + k] * vd;
      lv[D] += lF[1 + k] * u[1 + k];
    }
    lp += lF[1 + D];
    lv[D] += lF[E::IE] * (u[E::IE] + w.p);
    lu[E::IE] += lF[E::IE] * vd;
    lp += lF[E::IE] * vd;
  } else {
    const double ptot = fma(0.5, w.b2, w.p);
    const double Bd = w.B[D];
    const double bv = fma(w.B[2], w.v[2], fma(w.B[1], w.v[1], w.B[0] * w.v[0]));
    double lptot = 0.0, lbv = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lu[1 + k] += lF[1 + k] * vd;
      lv[D] += lF[1 + k] * u[1 + k];
      lB[D] += -lF[1 + k] * w.B[k];
      lB[k] += -lF[1 + k] * Bd;
    }
    lptot += lF[1 + D];
    lv[D] += lF[4] * (u[4] + ptot);
    lu[4] += lF[4] * vd;
    lptot += lF[4] * vd;
    lB[D] += -lF[4] * bv;
    lbv += -lF[4] * Bd;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k == D) continue;
      lv[D] += lF[5 + k] * w.B[k];
      lB[k] += lF[5 + k] * vd;
      lB[D] += -lF[5 + k] * w.v[k];
      lv[k] += -lF[5 + k] * Bd;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lB[k] += lbv * w.v[k];
      lv[k] += lbv * w.B[k];
    }
    lp += lptot;
    const double lb2 = 0.5 * lptot;
#pragma unroll
    for (int k = 0; k < 3; ++k) lB[k] += 2.0 * w.B[k] * lb2;
  }
  prim_vjp<NDIM, MHD>(u, w, gamma, lv, lp, 0.0, lB, lu);
}

// lu += ls * d(|v_d| + c_f,d)/dU   (d|v|/dv := 0 at v = 0).
template <int NDIM, bool MHD>
__device__ void speed_vjp(const double* u, double gamma, int d, double ls, double* lu) {
  PrimD w;
  prim<NDIM, MHD>(u, gamma, w);
  double lv[3] = {0.0, 0.0, 0.0}, lB[3] = {0.0, 0.0, 0.0};
  double lp = 0.0, lri = 0.0;
  lv[d] += (w.v[d] > 0.0) ? ls : (w.v[d] < 0.0 ? -ls : 0.0);
  const double a2 = gamma * w.p * w.ri;
  if constexpr (!MHD) {
    const double cs = sqrt(a2);
    const double la2 = ls / (2.0 * cs);
    lp += gamma * w.ri * la2;
    lri += gamma * w.p * la2;
  } else {
    const double b2n = w.b2 * w.ri;
    const double bd2 = w.B[d] * w.B[d] * w.ri;
    const double s = a2 + b2n;
    double disc = fma(s, s, -4.0 * a2 * bd2);
    const bool pos = disc > 0.0;
    disc = pos ? disc : 0.0;
    const double q = sqrt(disc);
    const double cf = sqrt(0.5 * (s + q));
    const double lcf2 = ls / (2.0 * cf);
    double lS = 0.5 * lcf2;
    const double lq = 0.5 * lcf2;
    const double ldisc = pos ? lq / (2.0 * q) : 0.0;
    lS += 2.0 * s * ldisc;
    double la2 = -4.0 * bd2 * ldisc + lS;
    const double lbd2 = -4.0 * a2 * ldisc;
    const double lb2n = lS;
    lp += gamma * w.ri * la2;
    lri += gamma * w.p * la2;
    const double lb2 = w.ri * lb2n;
    lri += w.b2 * lb2n;
    lB[d] += 2.0 * w.B[d] * w.ri * lbd2;
    lri += w.B[d] * w.B[d] * lbd2;
#pragma unroll
    for (int k = 0; k < 3; ++k) lB[k] += 2.0 * w.B[k] * lb2;
  }
  prim_vjp<NDIM, MHD>(u, w, gamma, lv, lp, lri, lB, lu);
}

template <int TX, int TY, int TZ>
struct AdjShape {
  static constexpr int T(int d) { return d == 0 ? TX : d == 1 ? TY : TZ; }
  static constexpr int TC = TX * TY * TZ;
  static constexpr int EF(int D, int d) { return T(d) + (d == D ? 10 : 0); }   // F+-: cells o-5 .. o+T+4
  static constexpr int NF(int D) { return EF(D, 0) * EF(D, 1) * EF(D, 2); }
  static constexpr int SF(int D) { return D == 0 ? 1 : D == 1 ? EF(D, 0) : EF(D, 0) * EF(D, 1); }
  static constexpr int EM(int D, int d) { return T(d) + (d == D ? 6 : 0); }    // mu: cells o-3 .. o+T+2
  static constexpr int NM(int D) { return EM(D, 0) * EM(D, 1) * EM(D, 2); }
  static constexpr int SM(int D) { return D == 0 ? 1 : D == 1 ? EM(D, 0) : EM(D, 0) * EM(D, 1); }
  static constexpr int EI(int D, int d) { return T(d) + (d == D ? 5 : 0); }    // interfaces o-3 .. o+T+1 (+1/2)
  static constexpr int NI(int D) { return EI(D, 0) * EI(D, 1) * EI(D, 2); }
  static constexpr int SI(int D) { return D == 0 ? 1 : D == 1 ? EI(D, 0) : EI(D, 0) * EI(D, 1); }
};

template <int NDIM, bool MHD, int TX, int TY, int TZ, int NT, int NGRP>
__global__ void __launch_bounds__(NT) k_vjp(VjpParams P) {
  using E = Eq<NDIM, MHD>;
  using S = AdjShape<TX, TY, TZ>;
  constexpr int NV = E::NV;
  constexpr int VPG = (NV + NGRP - 1) / NGRP;
  constexpr int TC = S::TC;
  constexpr int CPT = (TC + NT - 1) / NT;
  constexpr int NFM = cmax_i<cmax_i<S::NF(0), NDIM >= 2 ? S::NF(1) : 0>::v, NDIM >= 3 ? S::NF(2) : 0>::v;
  constexpr int NMM = cmax_i<cmax_i<S::NM(0), NDIM >= 2 ? S::NM(1) : 0>::v, NDIM >= 3 ? S::NM(2) : 0>::v;
  constexpr int NIM = cmax_i<cmax_i<S::NI(0), NDIM >= 2 ? S::NI(1) : 0>::v, NDIM >= 3 ? S::NI(2) : 0>::v;
  __shared__ double sF[2 * VPG * NFM];
  __shared__ double sMu[VPG * NMM];
  __shared__ double sLF[VPG * NIM];
  __shared__ unsigned char sCP[VPG * NIM];
  __shared__ unsigned char sCM[VPG * NIM];
  __shared__ double red[NT / 64][3];

  const int tid = threadIdx.x;
  const StateTable& st = P.st;
  const double gamma = P.gamma;
  double cin[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) cin[d] = __longlong_as_double((long long)P.ctl->cm[P.cm_slot][d]);

  const TileSchedule sched(P.ntiles);
  for (int t = sched.t; t < sched.end; t += sched.step) {
    const Tile tl = P.tiles[t];
    const BlockDev& B = st.blocks[tl.block];
    int tend[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int rem = B.n[d] - tl.o[d];
      tend[d] = rem < S::T(d) ? rem : S::T(d);
    }
    // owned cells: state, primitives, accumulators
    double uo[CPT][NV];
    PrimD wo[CPT];
    double nu[CPT][NV];
    bool own[CPT];
    double cp[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      const int cidx = tid + r * NT;
      int a0 = cidx % TX, a1 = (cidx / TX) % TY, a2 = cidx / (TX * TY);
      own[r] = cidx < TC && a0 < tend[0] && a1 < tend[1] && a2 < tend[2];
#pragma unroll
      for (int v = 0; v < NV; ++v) nu[r][v] = 0.0;
      if (own[r]) {
        long long vs;
        const double* p = cell_addr(st, B, P.in, tl.o[0] + a0, tl.o[1] + a1, tl.o[2] + a2, vs);
#pragma unroll
        for (int v = 0; v < NV; ++v) uo[r][v] = p[v * vs];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) uo[r][v] = (v == 0) ? 1.0 : 0.0;
        uo[r][E::IE] = 1.0;
      }
      prim<NDIM, MHD>(uo[r], gamma, wo[r]);
    }

    static_for<0, NDIM>([&](auto Dc) {
      constexpr int D = decltype(Dc)::value;
      constexpr int NF_D = S::NF(D), NM_D = S::NM(D), NI_D = S::NI(D);
      constexpr int F0 = S::EF(D, 0), F1 = S::EF(D, 1);
      constexpr int M0 = S::EM(D, 0), M1 = S::EM(D, 1);
      constexpr int I0 = S::EI(D, 0), I1 = S::EI(D, 1);
      constexpr int SFD = S::SF(D), SMD = S::SM(D), SID = S::SI(D);
      const double c = cin[D];
      const double idx_d = B.inv_dx[D];

      static_for<0, NGRP>([&](auto Gc) {
        constexpr int G = decltype(Gc)::value;
        constexpr int V0 = G * VPG;
        constexpr int VN = (V0 + VPG <= NV) ? VPG : NV - V0;
        // A) split fluxes on o-5 .. o+T+4 and mu on o-3 .. o+T+2 along D
        for (int e = tid; e < NF_D; e += NT) {
          int a[3] = {e % F0, (e / F0) % F1, e / (F0 * F1)};
          bool valid = true;
          int cc[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            valid = valid && (a[d] < tend[d] + (d == D ? 10 : 0));
            cc[d] = tl.o[d] + a[d] - (d == D ? 5 : 0);
          }
          if (valid) {
            double u[NV];
            load_cell<NV, D>(st, tl.block, P.in, cc[0], cc[1], cc[2], u);
            PrimD w;
            prim<NDIM, MHD>(u, gamma, w);
            double F[NV];
            phys_flux<NDIM, MHD, D>(u, w, F);
#pragma unroll
            for (int vg = 0; vg < VN; ++vg) {
              sF[vg * NF_D + e] = 0.5 * fma(c, u[V0 + vg], F[V0 + vg]);
              sF[(VPG + vg) * NF_D + e] = 0.5 * fma(-c, u[V0 + vg], F[V0 + vg]);
            }
          }
        }
        for (int m = tid; m < NM_D; m += NT) {
          int a[3] = {m % M0, (m / M0) % M1, m / (M0 * M1)};
          bool valid = true;
          int cc[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            valid = valid && (a[d] < tend[d] + (d == D ? 6 : 0));
            cc[d] = tl.o[d] + a[d] - (d == D ? 3 : 0);
          }
          if (valid) {
            double mu[VN];
            load_cell_vars<V0, VN, D>(st, tl.block, P.mu, cc[0], cc[1], cc[2], mu);
#pragma unroll
            for (int vg = 0; vg < VN; ++vg) sMu[vg * NM_D + m] = mu[vg];
          }
        }
        __syncthreads();
        // B) interface adjoints and MP5 pieces
        for (int wi = tid; wi < VN * NI_D; wi += NT) {
          const int vg = wi / NI_D;
          const int q = wi - vg * NI_D;
          int a[3] = {q % I0, (q / I0) % I1, q / (I0 * I1)};
          bool valid = true;
#pragma unroll
          for (int d = 0; d < 3; ++d) valid = valid && (a[d] < tend[d] + (d == D ? 5 : 0));
          if (!valid) continue;
          // stencil cells i-2 .. i+3 are F-box indices a_D .. a_D + 5 along D
          const int eb = a[0] + F0 * (a[1] + F1 * a[2]);
          const double* fp = &sF[vg * NF_D + eb];
          const double* fm = &sF[(VPG + vg) * NF_D + eb];
          sCP[vg * NI_D + q] = (unsigned char)mp5_code(fp[0], fp[SFD], fp[2 * SFD], fp[3 * SFD], fp[4 * SFD]);
          sCM[vg * NI_D + q] = (unsigned char)mp5_code(fm[5 * SFD], fm[4 * SFD], fm[3 * SFD], fm[2 * SFD], fm[SFD]);
          // mu_i and mu_{i+1} are mu-box indices a_D and a_D + 1 along D
          const int mb = a[0] + M0 * (a[1] + M1 * a[2]);
          sLF[vg * NI_D + q] = (sMu[vg * NM_D + mb + SMD] - sMu[vg * NM_D + mb]) * idx_d;
        }
        __syncthreads();
        // C) gather into the owned cells
#pragma unroll
        for (int r = 0; r < CPT; ++r) {
          if (!own[r]) continue;
          const int cidx = tid + r * NT;
          const int a0 = cidx % TX, a1 = (cidx / TX) % TY, a2 = cidx / (TX * TY);
          const int ib = a0 + I0 * (a1 + I1 * a2);
          double lF[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) lF[v] = 0.0;
#pragma unroll
          for (int vg = 0; vg < VN; ++vg) {
            const double* lf = &sLF[vg * NI_D + ib];
            const unsigned char* kp = &sCP[vg * NI_D + ib];
            const unsigned char* km = &sCM[vg * NI_D + ib];
            double lm = 0.0, lp = 0.0;
#pragma unroll
            for (int s = 0; s <= 4; ++s) lm = fma(lf[s * SID], c_mp5w[km[s * SID]][s], lm);
#pragma unroll
            for (int s = 1; s <= 5; ++s) lp = fma(lf[s * SID], c_mp5w[kp[s * SID]][5 - s], lp);
            const int v = V0 + vg;
            lF[v] = 0.5 * (lp + lm);
            nu[r][v] = fma(0.5 * c, lp - lm, nu[r][v]);
            cp[D] = fma(0.5 * uo[r][v], lp - lm, cp[D]);
          }
          flux_vjp<NDIM, MHD, D>(uo[r], wo[r], gamma, lF, nu[r]);
        }
        __syncthreads();
      });
    });

    // lam += scale * nu
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      if (!own[r]) continue;
      const int cidx = tid + r * NT;
      const int a0 = cidx % TX, a1 = (cidx / TX) % TY, a2 = cidx / (TX * TY);
      long long vs;
      double* p = const_cast<double*>(cell_addr(st, B, P.lam, tl.o[0] + a0, tl.o[1] + a1, tl.o[2] + a2, vs));
#pragma unroll
      for (int v = 0; v < NV; ++v) p[v * vs] = fma(P.scale, nu[r][v], p[v * vs]);
    }
    // per-tile c_max adjoint sums (fixed reduction order)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double x = cp[d];
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
      cp[d] = x;
    }
    if ((tid & 63) == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) red[tid >> 6][d] = cp[d];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double x = red[0][d];
        for (int q = 1; q < NT / 64; ++q) x += red[q][d];
        P.cpart[3 * (long long)t + d] = x;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// c_max with its maximising cell: per tile, then one work-group.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool better(double v, long long k, double bv, long long bk) {
  return v > bv || (v == bv && k < bk);
}

template <int NDIM, bool MHD>
__global__ void __launch_bounds__(256) k_argmax_tiles(StateTable st, const Tile* tiles, int ntiles, int tx, int ty,
                                                      int tz, double gamma, int in, double* tmax, long long* targ) {
  using E = Eq<NDIM, MHD>;
  __shared__ double sv[256][3];
  __shared__ long long sk[256][3];
  const int tid = threadIdx.x;
  const int tcells = tx * ty * tz;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile tl = tiles[t];
    const BlockDev& B = st.blocks[tl.block];
    double bv[3] = {-1.0, -1.0, -1.0};
    long long bk[3] = {0x7fffffffffffffffll, 0x7fffffffffffffffll, 0x7fffffffffffffffll};
    for (int c = tid; c < tcells; c += 256) {
      const int i = tl.o[0] + c % tx, j = tl.o[1] + (c / tx) % ty, k = tl.o[2] + c / (tx * ty);
      if (i >= B.n[0] || j >= B.n[1] || k >= B.n[2]) continue;
      long long vs;
      const double* p = cell_addr(st, B, in, i, j, k, vs);
      double u[E::NV];
#pragma unroll
      for (int v = 0; v < E::NV; ++v) u[v] = p[v * vs];
      PrimD w;
      prim<NDIM, MHD>(u, gamma, w);
      const long long key = ((long long)tl.block << 32) | (long long)(((long long)k * B.n[1] + j) * B.n[0] + i);
#pragma unroll
      for (int d = 0; d < NDIM; ++d) {
        const double s = fabs(w.v[d]) + fast_speed<MHD>(w, d, gamma);
        if (better(s, key, bv[d], bk[d])) { bv[d] = s; bk[d] = key; }
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) { sv[tid][d] = bv[d]; sk[tid][d] = bk[d]; }
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
      if (tid < h) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
          if (better(sv[tid + h][d], sk[tid + h][d], sv[tid][d], sk[tid][d])) {
            sv[tid][d] = sv[tid + h][d];
            sk[tid][d] = sk[tid + h][d];
          }
      }
      __syncthreads();
    }
    if (tid == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) { tmax[3 * (long long)t + d] = sv[0][d]; targ[3 * (long long)t + d] = sk[0][d]; }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_argmax_reduce(const double* tmax, const long long* targ, int ntiles,
                                                       Control* ctl, int slot) {
  __shared__ double sv[256][3];
  __shared__ long long sk[256][3];
  const int tid = threadIdx.x;
  double bv[3] = {-1.0, -1.0, -1.0};
  long long bk[3] = {0x7fffffffffffffffll, 0x7fffffffffffffffll, 0x7fffffffffffffffll};
  for (int t = tid; t < ntiles; t += 256)
    for (int d = 0; d < 3; ++d)
      if (better(tmax[3 * (long long)t + d], targ[3 * (long long)t + d], bv[d], bk[d])) {
        bv[d] = tmax[3 * (long long)t + d];
        bk[d] = targ[3 * (long long)t + d];
      }
  for (int d = 0; d < 3; ++d) { sv[tid][d] = bv[d]; sk[tid][d] = bk[d]; }
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h)
      for (int d = 0; d < 3; ++d)
        if (better(sv[tid + h][d], sk[tid + h][d], sv[tid][d], sk[tid][d])) {
          sv[tid][d] = sv[tid + h][d];
          sk[tid][d] = sk[tid + h][d];
        }
    __syncthreads();
  }
  if (tid == 0)
    for (int d = 0; d < 3; ++d) {
      const double m = sv[0][d] < 0.0 ? 0.0 : sv[0][d];
      ctl->cm[slot][d] = (unsigned long long)__double_as_longlong(m);
      ctl->arg[d] = sk[0][d];
    }
}

// Sum of the per-tile c_max adjoints (fixed order), then
// lam[argmax_d] += scale * lamc_d * d(|v_d| + c_f,d)/dU at the maximiser.
template <int NDIM, bool MHD>
__global__ void __launch_bounds__(256) k_vjp_cmax(StateTable st, int nblocks, const double* cpart, int ntiles,
                                                  Control* ctl, double gamma, int in, int lam, double scale) {
  using E = Eq<NDIM, MHD>;
  __shared__ double s[256][3];
  const int tid = threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int t = tid; t < ntiles; t += 256)
    for (int d = 0; d < 3; ++d) acc[d] += cpart[3 * (long long)t + d];
  for (int d = 0; d < 3; ++d) s[tid][d] = acc[d];
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h)
      for (int d = 0; d < 3; ++d) s[tid][d] += s[tid + h][d];
    __syncthreads();
  }
  if (tid != 0) return;
  for (int d = 0; d < NDIM; ++d) {
    const long long key = ctl->arg[d];
    const int b = (int)(key >> 32);
    const long long cell = key & 0xffffffffll;
    // no cell had a finite speed (non-physical state): report, never index
    if (key < 0 || b < 0 || b >= nblocks) {
      atomicOr(&ctl->err, 1);
      return;
    }
    const BlockDev& B = st.blocks[b];
    if (cell >= B.cells) {
      atomicOr(&ctl->err, 1);
      return;
    }
    const int i = (int)(cell % B.n[0]), j = (int)((cell / B.n[0]) % B.n[1]), k = (int)(cell / ((long long)B.n[0] * B.n[1]));
    long long vs, ws;
    const double* p = cell_addr(st, B, in, i, j, k, vs);
    double u[E::NV], lu[E::NV];
    for (int v = 0; v < E::NV; ++v) {
      u[v] = p[v * vs];
      lu[v] = 0.0;
    }
    speed_vjp<NDIM, MHD>(u, gamma, d, s[0][d], lu);
    double* q = const_cast<double*>(cell_addr(st, B, lam, i, j, k, ws));
    for (int v = 0; v < E::NV; ++v) q[v * ws] = fma(scale, lu[v], q[v * ws]);
  }
}

// dst = sum_j a[j] * src[j] over the interiors (up to 6 terms; dst may be a
// source).
struct CombineParams {
  StateTable st;
  const Tile* tiles;
  int ntiles, tx, ty, tz, nv;
  int n;
  int src[6];
  double a[6];
  int dst;
};

__global__ void __launch_bounds__(256) k_combine(CombineParams P) {
  const int tcells = P.tx * P.ty * P.tz;
  for (int t = blockIdx.x; t < P.ntiles; t += gridDim.x) {
    const Tile tl = P.tiles[t];
    const BlockDev& B = P.st.blocks[tl.block];
    for (int c = threadIdx.x; c < tcells; c += 256) {
      const int i = tl.o[0] + c % P.tx, j = tl.o[1] + (c / P.tx) % P.ty, k = tl.o[2] + c / (P.tx * P.ty);
      if (i >= B.n[0] || j >= B.n[1] || k >= B.n[2]) continue;
      long long vs[6], ws;
      const double* sp[6];
      for (int q = 0; q < P.n; ++q) sp[q] = cell_addr(P.st, B, P.src[q], i, j, k, vs[q]);
      double* dp = const_cast<double*>(cell_addr(P.st, B, P.dst, i, j, k, ws));
      for (int v = 0; v < P.nv; ++v) {
        double acc = 0.0;
        for (int q = 0; q < P.n; ++q) acc = fma(P.a[q], sp[q][v * vs[q]], acc);
        dp[v * ws] = acc;
      }
    }
  }
}

// Caller's padded lambda arrays <-> scratch slot (interior).  Export writes
// zeros into the ghost layers.
__global__ void __launch_bounds__(256) k_lam_import(StateTable st, double* const* ptrs, int nv, int dst) {
  const int b = blockIdx.x;
  const BlockDev& B = st.blocks[b];
  for (long long c = threadIdx.x; c < B.cells; c += 256) {
    const int i = (int)(c % B.n[0]), j = (int)((c / B.n[0]) % B.n[1]), k = (int)(c / ((long long)B.n[0] * B.n[1]));
    const long long pstride = (long long)B.P[0] * B.P[1] * B.P[2];
    const long long pidx = ((long long)(k + B.g[2]) * B.P[1] + (j + B.g[1])) * B.P[0] + (i + B.g[0]);
    long long ws;
    double* q = const_cast<double*>(cell_addr(st, B, dst, i, j, k, ws));
    for (int v = 0; v < nv; ++v) q[v * ws] = ptrs[b][v * pstride + pidx];
  }
}

__global__ void __launch_bounds__(256) k_lam_export(StateTable st, double* const* ptrs, int nv, int src) {
  const int b = blockIdx.x;
  const BlockDev& B = st.blocks[b];
  const long long pstride = (long long)B.P[0] * B.P[1] * B.P[2];
  for (long long pc = threadIdx.x; pc < pstride; pc += 256) {
    const int pi = (int)(pc % B.P[0]), pj = (int)((pc / B.P[0]) % B.P[1]), pk = (int)(pc / ((long long)B.P[0] * B.P[1]));
    const int i = pi - B.g[0], j = pj - B.g[1], k = pk - B.g[2];
    const bool inside = i >= 0 && i < B.n[0] && j >= 0 && j < B.n[1] && k >= 0 && k < B.n[2];
    if (inside) {
      long long vs;
      const double* p = cell_addr(st, B, src, i, j, k, vs);
      for (int v = 0; v < nv; ++v) ptrs[b][v * pstride + pc] = p[v * vs];
    } else {
      for (int v = 0; v < nv; ++v) ptrs[b][v * pstride + pc] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
struct VjpVariant {
  int ndim, mhd, tx, ty, tz, nt;
  const void* fn;
  void (*launch)(const VjpParams&, int grid, hipStream_t);
  void (*argmax)(StateTable, const Tile*, int, int, int, int, double, int, double*, long long*, int, hipStream_t);
  void (*cmax_term)(StateTable, int, const double*, int, Control*, double, int, int, double, hipStream_t);
};

template <int NDIM, bool MHD, int TX, int TY, int TZ, int NT, int NGRP>
static void launch_vjp_t(const VjpParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_vjp<NDIM, MHD, TX, TY, TZ, NT, NGRP>), dim3(grid), dim3(NT), 0, s, p);
}

template <int NDIM, bool MHD>
static void launch_argmax_t(StateTable st, const Tile* tiles, int ntiles, int tx, int ty, int tz, double gamma,
                            int in, double* tmax, long long* targ, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_argmax_tiles<NDIM, MHD>), dim3(grid), dim3(256), 0, s, st, tiles, ntiles, tx, ty, tz, gamma,
                     in, tmax, targ);
}

template <int NDIM, bool MHD>
static void launch_cmax_term_t(StateTable st, int nblocks, const double* cpart, int ntiles, Control* ctl, double gamma,
                               int in, int lam, double scale, hipStream_t s) {
  hipLaunchKernelGGL((k_vjp_cmax<NDIM, MHD>), dim3(1), dim3(256), 0, s, st, nblocks, cpart, ntiles, ctl, gamma, in,
                     lam, scale);
}

#define AMRVAC_VJP(ND, M, TX, TY, TZ, NT, NGRP)                                                          \
  {ND, M, TX, TY, TZ, NT, (const void*)&k_vjp<ND, M, TX, TY, TZ, NT, NGRP>,                               \
   &launch_vjp_t<ND, M, TX, TY, TZ, NT, NGRP>, &launch_argmax_t<ND, M>, &launch_cmax_term_t<ND, M>}

static const VjpVariant g_vjp[] = {
    AMRVAC_VJP(1, false, 64, 1, 1, 64, 1),
    AMRVAC_VJP(1, true, 64, 1, 1, 64, 2),
    AMRVAC_VJP(2, false, 16, 16, 1, 256, 1),
    AMRVAC_VJP(2, true, 16, 16, 1, 256, 2),
    AMRVAC_VJP(3, false, 8, 8, 4, 256, 3),
    AMRVAC_VJP(3, true, 8, 8, 4, 256, 4),
};

const VjpVariant* vjp_variant(int ndim, int mhd) {
  for (const VjpVariant& v : g_vjp)
    if (v.ndim == ndim && v.mhd == mhd) return &v;
  return nullptr;
}

void launch_argmax_reduce(const double* tmax, const long long* targ, int ntiles, Control* ctl, int slot,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_argmax_reduce, dim3(1), dim3(256), 0, s, tmax, targ, ntiles, ctl, slot);
}

void launch_combine(const CombineParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(grid), dim3(256), 0, s, p);
}

void launch_lam_import(StateTable st, double* const* ptrs, int nv, int dst, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_lam_import, dim3(nblocks), dim3(256), 0, s, st, ptrs, nv, dst);
}

void launch_lam_export(StateTable st, double* const* ptrs, int nv, int src, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_lam_export, dim3(nblocks), dim3(256), 0, s, st, ptrs, nv, src);
}

}  // namespace amrvac
