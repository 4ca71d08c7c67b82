// Reverse mode of the FD-MP5 / global-LF right-hand side (Porth et al. 2014,
// Sects. 2.1-2.2) on gfx950, used by the adjoint of the SSPRK time
// integration (Sect. 2.3).
//
// k_vjp computes dst = sum_q a_q lam_q + scale * J_L(U)^T mu for the local
// dependence of L on U (everything but the global c_max), as a gather per
// cell so that no atomics are needed and the result is deterministic.  MP5
// with eps = 0 is continuous and piecewise linear, so its derivative at U is
// one of 14 constant weight vectors per reconstruction; LIM03 is piecewise
// linear too (5 pieces; its asymptotic-region switch is a jump on a set of
// measure zero, where the derivative of the branch taken is used).  The
// forward recompute of U's stage records the piece as a 4-bit code per
// (interface, variable, sign), and k_vjp reads those codes instead of
// re-evaluating the split fluxes and the limiter.  Per cell j and direction d:
//   lamFhat_{i+1/2} = (mu_{i+1} - mu_i) / dx_d,
//   lamF+_j = sum over interfaces i = j-2 .. j+2 of lamFhat w+_i,
//   lamF-_j = sum over interfaces i = j-3 .. j+1 of lamFhat w-_i,
// then the split adjoint (lamF = (lamF+ + lamF-)/2, c (lamF+ - lamF-)/2) and
// the transpose of the flux Jacobian (hand-written reverse of the primitive
// recovery and flux).
// The c_max term sum_j U_j (lamF+_j - lamF-_j)/2 is summed per work-group
// over its tiles; k_vjp_cmax adds the total's product with d(|v_d| +
// c_f,d)/dU at the maximising cell (lowest block, then lowest cell index, on
// ties).  On fixed faces, k_vjp_ghost forms the same split adjoint and flux
// transpose for the caller's ghost cells, the adjoint of the boundary data.
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

// Weights of the LIM03 inputs for each of its linear pieces, placed on the
// same five stencil positions (f_{j-2} .. f_{j+2}; LIM03 reads f_{j-1} ..
// f_{j+1}): 0 f_j; 1 the third-order formula (-f_{j-1} + 5 f_j + 2
// f_{j+1})/6; 2 phi = -theta/2; 3 phi = 2 theta; 4 phi = 1.6.
__constant__ double c_lim3w[5][5] = {
    {0.0, 0.0, 1.0, 0.0, 0.0},
    {0.0, -1.0 / 6.0, 5.0 / 6.0, 1.0 / 3.0, 0.0},
    {0.0, 0.25, 0.75, 0.0, 0.0},
    {0.0, -1.0, 2.0, 0.0, 0.0},
    {0.0, 0.0, 1.0 - 0.5 * 1.6, 0.5 * 1.6, 0.0},
};

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
struct SweepShape {
  static constexpr int T(int d) { return d == 0 ? TX : d == 1 ? TY : TZ; }
  static constexpr int TC = TX * TY * TZ;
  // pencils along D (the tile's cross-section), LDS row stride made odd
  static constexpr int NP(int D) { return TC / T(D); }
  static constexpr int PSTR(int D) { return NP(D) | 1; }
  // a sweep item covers SEG consecutive cells of one pencil: at most 8, and
  // halved (while it divides the pencil and stays >= 2) until the items of
  // NV variables fill NT threads, so that small-variable-count shapes keep
  // every thread busy with shorter walks
  static constexpr int SEG(int D, int NV, int NT) {
    int seg = T(D) < 8 ? T(D) : 8;
    while (seg > 2 && seg % 2 == 0 && NP(D) * NV * (T(D) / seg) < NT) seg /= 2;
    return seg;
  }
  // mu rows: cells o_D-3 .. o_D+T_D+2; code rows: lower faces of cells
  // o_D-2 .. o_D+T_D+2 (interfaces i+1/2, i = o_D-3 .. o_D+T_D+1)
  static constexpr int MROWS(int D) { return T(D) + 6; }
  static constexpr int CROWS(int D) { return T(D) + 5; }
  static constexpr int PENC(int D, int a0, int a1, int a2) {
    return D == 0 ? a1 + TY * a2 : D == 1 ? a0 + TX * a2 : a0 + TX * a1;
  }
};

// Cell (c[0], c[1], c[2]) of block blk where only c[D] may lie outside the
// block: the face neighbour that holds it, with c[D] moved into it (nullptr
// for a fixed face, which the adjoint rejects before any launch).
template <int D>
__device__ __forceinline__ const BlockDev* resolve_cell(const StateTable& st, int blk, int* c) {
  const BlockDev* B = &st.blocks[blk];
  if (c[D] < 0) {
    const int nb = B->nbr[2 * D];
    if (nb < 0) return nullptr;
    B = &st.blocks[nb];
    c[D] += B->n[D];
  } else if (c[D] >= B->n[D]) {
    const int nb = B->nbr[2 * D + 1];
    if (nb < 0) return nullptr;
    c[D] -= B->n[D];
    B = &st.blocks[nb];
  }
  return B;
}

// Per tile and direction D:
//   A) mu = sum_q mu_a[q] lam_q on the tile extended by 3 cells along D, and
//      the 8 code bytes of every interface the tile's cells depend on, into
//      LDS (rows along D, pencils contiguous);
//   B) one work item per (pencil, variable, segment of SEG cells) walks the
//      SEG + 5 interfaces that reach the segment: lamFhat = (mu_{i+1} -
//      mu_i)/dx, then lamF+ and lamF- of the cells in the interface's two
//      stencils += lamFhat * weight of the stencil position in the coded
//      piece, all in registers (each cell receives its terms in increasing
//      interface order);
//   C) per owned cell: split adjoint and flux transpose.
// Then dst = sum_q lam_a[q] lam_q + scale * nu for the owned cells.
template <int NDIM, bool MHD, int TX, int TY, int TZ, int NT>
__global__ void __launch_bounds__(NT) k_vjp(VjpParams P) {
  using E = Eq<NDIM, MHD>;
  using S = SweepShape<TX, TY, TZ>;
  constexpr int NV = E::NV;
  constexpr int TC = S::TC;
  constexpr int CPT = (TC + NT - 1) / NT;
  constexpr int MB = cmax_i<cmax_i<NV * S::MROWS(0) * S::PSTR(0), NDIM >= 2 ? NV * S::MROWS(1) * S::PSTR(1) : 0>::v,
                            NDIM >= 3 ? NV * S::MROWS(2) * S::PSTR(2) : 0>::v;
  constexpr int OB = cmax_i<cmax_i<2 * NV * S::T(0) * S::PSTR(0), NDIM >= 2 ? 2 * NV * S::T(1) * S::PSTR(1) : 0>::v,
                            NDIM >= 3 ? 2 * NV * S::T(2) * S::PSTR(2) : 0>::v;
  constexpr int CB = cmax_i<cmax_i<S::CROWS(0) * S::PSTR(0), NDIM >= 2 ? S::CROWS(1) * S::PSTR(1) : 0>::v,
                            NDIM >= 3 ? S::CROWS(2) * S::PSTR(2) : 0>::v;
  // mu box, reused for the sweep outputs once every item has read it
  __shared__ double sMu[cmax_i<MB, OB>::v];
  __shared__ unsigned long long sCode[CB];
  __shared__ double sW[16 * 5];
  __shared__ double red[NT / 64][3];

  const int tid = threadIdx.x;
  const StateTable& st = P.st;
  const double gamma = P.gamma;
  if (P.recon == 1) {
    for (int q = tid; q < 16 * 5; q += NT) sW[q] = q < 5 * 5 ? c_lim3w[q / 5][q % 5] : 0.0;
  } else {
    for (int q = tid; q < 16 * 5; q += NT) sW[q] = q < 14 * 5 ? c_mp5w[q / 5][q % 5] : 0.0;
  }
  double cin[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) cin[d] = P.cm_in[d];
  __syncthreads();
  // the piece almost every interface takes (MP5: the fifth-order value, code
  // 0; LIM03: the third-order formula, code 1), its weights in registers: a
  // wave whose interfaces all took it on both sides skips the table
  const int pc = P.recon == 1 ? 1 : 0;
  const int ccom = pc | (pc << 4);
  double wc[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) wc[q] = sW[pc * 5 + q];

  // c_max adjoint sums of this work-group's tiles (taken in the fixed tile
  // order of the schedule, then a fixed butterfly: deterministic)
  double cp[3] = {0.0, 0.0, 0.0};
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
    // owned cells: state, primitives, accumulators, mu (formed once per
    // tile; each direction then loads only the halo rows of mu) and the
    // lambda combination of the output.  Every load is issued first, term by
    // term over the thread's cells; primitives and the maximiser test follow.
    double uo[CPT][NV];
    PrimD wo[CPT];
    double nu[CPT][NV];
    double muo[CPT][NV];
    double acc[CPT][NV];
    bool own[CPT];
    int oc[CPT][3];
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      const int cidx = tid + r * NT;
      const int a0 = cidx % TX, a1 = (cidx / TX) % TY, a2 = cidx / (TX * TY);
      own[r] = cidx < TC && a0 < tend[0] && a1 < tend[1] && a2 < tend[2];
      oc[r][0] = tl.o[0] + a0;
      oc[r][1] = tl.o[1] + a1;
      oc[r][2] = tl.o[2] + a2;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        nu[r][v] = 0.0;
        muo[r][v] = 0.0;
        acc[r][v] = 0.0;
      }
      if (own[r]) {
        long long vs;
        gptr p = cell_addr(st, B, P.in, oc[r][0], oc[r][1], oc[r][2], vs);
#pragma unroll
        for (int v = 0; v < NV; ++v) uo[r][v] = p[v * vs];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) uo[r][v] = (v == 0) ? 1.0 : 0.0;
        uo[r][E::IE] = 1.0;
      }
    }
    for (int q = 0; q < P.nmu; ++q) {
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        if (!own[r]) continue;
        long long vs;
        gptr p = cell_addr(st, B, P.mu_src[q], oc[r][0], oc[r][1], oc[r][2], vs);
#pragma unroll
        for (int v = 0; v < NV; ++v) muo[r][v] = fma(P.mu_a[q], p[v * vs], muo[r][v]);
      }
    }
    for (int q = 0; q < P.nlam; ++q) {
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        if (!own[r]) continue;
        long long vs;
        gptr p = cell_addr(st, B, P.lam_src[q], oc[r][0], oc[r][1], oc[r][2], vs);
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[r][v] = fma(P.lam_a[q], p[v * vs], acc[r][v]);
      }
    }
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      prim<NDIM, MHD>(uo[r], gamma, wo[r]);
      if (own[r]) {
        // the cells that realise c_max (bitwise the speed the recompute
        // folded into it): the lowest key wins
        const long long key =
            ((long long)tl.block << 32) | (((long long)oc[r][2] * B.n[1] + oc[r][1]) * B.n[0] + oc[r][0]);
#pragma unroll
        for (int d = 0; d < NDIM; ++d)
          if (fabs(wo[r].v[d]) + fast_speed<MHD>(wo[r], d, gamma) == cin[d])
            atomicMin(reinterpret_cast<unsigned long long*>(&P.ctl->arg[d]), (unsigned long long)key);
      }
    }

    static_for<0, NDIM>([&](auto Dc) {
      constexpr int D = decltype(Dc)::value;
      constexpr int TD = S::T(D), NP = S::NP(D), PS = S::PSTR(D);
      constexpr int MR = S::MROWS(D), CR = S::CROWS(D);
      constexpr int SEG = S::SEG(D, NV, NT), NSEG = TD / SEG;
      constexpr int C0 = D == 0 ? CR : TX, C1 = D == 1 ? CR : TY, C2 = D == 2 ? CR : TZ;
      const double c = cin[D];
      const double idx_d = B.inv_dx[D];

      // A) mu on the extended box (owned cells from registers, the 3 + 3
      // halo rows along D from memory), codes on the interface box.  Every
      // load of this thread is issued first (codes, then the halo rows' mu,
      // term by term over all of this thread's halo cells); the owned cells'
      // mu goes to LDS while they are in flight.
      constexpr int NCB = C0 * C1 * C2, CPTC = (NCB + NT - 1) / NT;
      unsigned long long cw[CPTC];
      int cpos[CPTC];
#pragma unroll
      for (int r = 0; r < CPTC; ++r) {
        const int e = tid + r * NT;
        const int a[3] = {e % C0, (e / C0) % C1, e / (C0 * C1)};
        bool valid = e < NCB;
#pragma unroll
        for (int d = 0; d < 3; ++d) valid = valid && a[d] < tend[d] + (d == D ? 5 : 0);
        cw[r] = 0ull;
        cpos[r] = valid ? a[D] * PS + S::PENC(D, a[0], a[1], a[2]) : -1;
        if (!valid) continue;
        int cc[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) cc[d] = tl.o[d] + a[d] - (d == D ? 2 : 0);
        const int up = cc[D];   // before resolve_cell moves it into a neighbour
        const BlockDev* Bn = resolve_cell<D>(st, tl.block, cc);
        if (!Bn && up == B.n[D] && B.fco[D] >= 0) {
          // the interface on a fixed upper face: its word after the interior cells
          const long long tr = D == 0 ? (long long)cc[1] + (long long)B.n[1] * cc[2]
                             : D == 1 ? (long long)cc[0] + (long long)B.n[0] * cc[2]
                                      : (long long)cc[0] + (long long)B.n[0] * cc[1];
          cw[r] = *(__attribute__((address_space(1))) const unsigned long long*)(P.codes + D * P.code_plane +
                                                                                (P.code_faces + B.fco[D] + tr) * 8);
        }
        if (Bn) {
          const long long cell = ((long long)cc[2] * Bn->n[1] + cc[1]) * Bn->n[0] + cc[0];
          cw[r] = *(__attribute__((address_space(1))) const unsigned long long*)(P.codes + D * P.code_plane +
                                                                                (Bn->coff + cell) * 8);
        }
      }
      constexpr int H0 = D == 0 ? 6 : TX, H1 = D == 1 ? 6 : TY, H2 = D == 2 ? 6 : TZ;
      constexpr int NHB = H0 * H1 * H2, HPTM = (NHB + NT - 1) / NT;
      double hm[HPTM][NV];
      int hrow[HPTM], hpen[HPTM];
      const BlockDev* hB[HPTM];
      int hc[HPTM][3];
#pragma unroll
      for (int r = 0; r < HPTM; ++r) {
        const int e = tid + r * NT;
        int a[3] = {e % H0, (e / H0) % H1, e / (H0 * H1)};
        bool valid = e < NHB;
#pragma unroll
        for (int d = 0; d < 3; ++d)
          if (d != D) valid = valid && a[d] < tend[d];
        if (a[D] >= 3) a[D] += tend[D];   // rows 0..2 below the tile, tend+3 .. tend+5 above
#pragma unroll
        for (int d = 0; d < 3; ++d) hc[r][d] = tl.o[d] + a[d] - (d == D ? 3 : 0);
        hB[r] = valid ? resolve_cell<D>(st, tl.block, hc[r]) : nullptr;
        hrow[r] = valid ? a[D] : -1;
        hpen[r] = S::PENC(D, a[0], a[1], a[2]);
#pragma unroll
        for (int v = 0; v < NV; ++v) hm[r][v] = 0.0;
      }
      for (int q = 0; q < P.nmu; ++q) {
#pragma unroll
        for (int r = 0; r < HPTM; ++r) {
          if (!hB[r]) continue;
          long long vs;
          gptr p = cell_addr(st, *hB[r], P.mu_src[q], hc[r][0], hc[r][1], hc[r][2], vs);
#pragma unroll
          for (int v = 0; v < NV; ++v) hm[r][v] = fma(P.mu_a[q], p[v * vs], hm[r][v]);
        }
      }
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        if (!own[r]) continue;
        const int cidx = tid + r * NT;
        int a[3] = {cidx % TX, (cidx / TX) % TY, cidx / (TX * TY)};
        const int pen = S::PENC(D, a[0], a[1], a[2]);
        const int row = a[D] + 3;
#pragma unroll
        for (int v = 0; v < NV; ++v) sMu[(v * MR + row) * PS + pen] = muo[r][v];
      }
#pragma unroll
      for (int r = 0; r < HPTM; ++r) {
        if (hrow[r] < 0) continue;
#pragma unroll
        for (int v = 0; v < NV; ++v) sMu[(v * MR + hrow[r]) * PS + hpen[r]] = hm[r][v];
      }
#pragma unroll
      for (int r = 0; r < CPTC; ++r)
        if (cpos[r] >= 0) sCode[cpos[r]] = cw[r];
      __syncthreads();

      // B) sweeps
      constexpr int NITEM = NP * NV * NSEG;
      constexpr int IPT = (NITEM + NT - 1) / NT;
      double rp[IPT][SEG], rm[IPT][SEG];
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const int item = tid + r * NT;
#pragma unroll
        for (int j = 0; j < SEG; ++j) { rp[r][j] = 0.0; rm[r][j] = 0.0; }
        if (item < NITEM) {
          const int pen = item % NP;
          const int v = (item / NP) % NV;
          const int g = item / (NP * NV);
          const double* mu = &sMu[(v * MR) * PS + pen];
          const unsigned char* cd = reinterpret_cast<const unsigned char*>(&sCode[pen]) + v;
          // every interface of the window on the common piece on both
          // sides, in every lane of the wave: the register weights serve
          bool common = true;
#pragma unroll
          for (int kk = 0; kk < SEG + 5; ++kk) common = common && cd[(g * SEG + kk) * PS * 8] == ccom;
          double mprev = mu[(g * SEG) * PS];
          if (__ballot(!common) == 0) {
#pragma unroll
            for (int kk = 0; kk < SEG + 5; ++kk) {
              const int k = g * SEG + kk;
              const double mnext = mu[(k + 1) * PS];
              const double lf = (mnext - mprev) * idx_d;
              mprev = mnext;
#pragma unroll
              for (int s = 0; s < 5; ++s) {
                const int j = kk - 5 + s;   // F+ stencil: cell i-2+s
                if (j >= 0 && j < SEG) rp[r][j] = fma(lf, wc[s], rp[r][j]);
              }
#pragma unroll
              for (int s = 0; s < 5; ++s) {
                const int j = kk - s;       // F- stencil: cell i+3-s
                if (j >= 0 && j < SEG) rm[r][j] = fma(lf, wc[s], rm[r][j]);
              }
            }
          } else {
#pragma unroll
            for (int kk = 0; kk < SEG + 5; ++kk) {
              const int k = g * SEG + kk;
              const double mnext = mu[(k + 1) * PS];
              const double lf = (mnext - mprev) * idx_d;
              mprev = mnext;
              const int code = cd[k * PS * 8];
              const double* wp = &sW[(code & 15) * 5];
              const double* wm = &sW[(code >> 4) * 5];
#pragma unroll
              for (int s = 0; s < 5; ++s) {
                const int j = kk - 5 + s;
                if (j >= 0 && j < SEG) rp[r][j] = fma(lf, wp[s], rp[r][j]);
              }
#pragma unroll
              for (int s = 0; s < 5; ++s) {
                const int j = kk - s;
                if (j >= 0 && j < SEG) rm[r][j] = fma(lf, wm[s], rm[r][j]);
              }
            }
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const int item = tid + r * NT;
        if (item < NITEM) {
          const int pen = item % NP;
          const int v = (item / NP) % NV;
          const int g = item / (NP * NV);
#pragma unroll
          for (int j = 0; j < SEG; ++j) {
            const int row = g * SEG + j;
            sMu[((0 * NV + v) * TD + row) * PS + pen] = 0.5 * (rp[r][j] + rm[r][j]);
            sMu[((1 * NV + v) * TD + row) * PS + pen] = rp[r][j] - rm[r][j];
          }
        }
      }
      __syncthreads();

      // C) split adjoint and flux transpose per owned cell
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        if (!own[r]) continue;
        const int cidx = tid + r * NT;
        const int a[3] = {cidx % TX, (cidx / TX) % TY, cidx / (TX * TY)};
        const int base = a[D] * PS + S::PENC(D, a[0], a[1], a[2]);
        double lF[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          lF[v] = sMu[(0 * NV + v) * TD * PS + base];
          const double dF = sMu[(1 * NV + v) * TD * PS + base];
          nu[r][v] = fma(0.5 * c, dF, nu[r][v]);
          cp[D] = fma(0.5 * uo[r][v], dF, cp[D]);
        }
        flux_vjp<NDIM, MHD, D>(uo[r], wo[r], gamma, lF, nu[r]);
      }
      __syncthreads();
    });

    // dst = sum_q lam_a[q] lam_q + scale * nu
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      if (!own[r]) continue;
      long long ws;
      gptr_w p = cell_addr_w(st, B, P.dst, oc[r][0], oc[r][1], oc[r][2], ws);
#pragma unroll
      for (int v = 0; v < NV; ++v) p[v * ws] = fma(P.scale, nu[r][v], acc[r][v]);
    }
  }
  // per-work-group c_max adjoint sums
#pragma unroll
  for (int d = 0; d < 3; ++d) cp[d] = wave_sum(cp[d]);
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
      P.cpart[3 * (long long)blockIdx.x + d] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the boundary data: the ghost cells of fixed faces.
// ---------------------------------------------------------------------------
// Weight of the stencil value at position s (0..4, f_{j-2} .. f_{j+2}) in
// the linear piece `code` of the reconstruction (MP5 or LIM03).
__device__ __forceinline__ double piece_weight(int recon, int code, int s) {
  return recon == 1 ? c_lim3w[code][s] : c_mp5w[code][s];
}

// For every face ghost cell g of the fixed faces, gadj[g] += scale *
// (dL/dU_g)^T mu: the interfaces i+1/2 (i = -1 .. n-1 of the block along the
// face's direction) whose F+ or F- stencil reaches g, through the linear
// pieces the recompute coded, then the split adjoint and the transpose of
// the flux at the ghost state (the caller's ghost values).  The ghost
// cells' share of the c_max adjoint goes to cpart[3 * blockIdx.x + d].
// One work-group per fixed face at a time (grid stride over faces).
template <int NDIM, bool MHD>
__global__ void __launch_bounds__(256) k_vjp_ghost(VjpParams P, const FixedFace* faces, int nfaces, double* gadj,
                                                   long long gplane, double* cpart) {
  using E = Eq<NDIM, MHD>;
  constexpr int NV = E::NV;
  __shared__ double red[4][3];
  const int tid = threadIdx.x;
  const StateTable& st = P.st;
  double cin[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) cin[d] = P.cm_in[d];
  double cp[3] = {0.0, 0.0, 0.0};
  for (int fi = blockIdx.x; fi < nfaces; fi += gridDim.x) {
    const FixedFace F = faces[fi];
    const BlockDev& B = st.blocks[F.block];
    const int D = F.face >> 1, side = F.face & 1;
    const int e0 = D == 0 ? 1 : 0, e1 = D == 2 ? 1 : 2;   // transverse directions, in order
    const int nt0 = B.n[e0], nt1 = B.n[e1];
    const long long area = (long long)nt0 * nt1;
    const int nD = B.n[D];
    const double idx_d = B.inv_dx[D];
    const double c = cin[D];
    for (long long q = tid; q < 3 * area; q += 256) {
      const int layer = (int)(q / area);
      const long long tr = q % area;
      int cc[3];
      cc[e0] = (int)(tr % nt0);
      cc[e1] = (int)(tr / nt0);
      const int m = side == 0 ? -1 - layer : nD + layer;   // the ghost cell along D
      // mu along the pencil (0 outside the interior)
      auto mu_at = [&](int j, int v) {
        if (j < 0 || j >= nD) return 0.0;
        int p3[3] = {cc[0], cc[1], cc[2]};
        p3[D] = j;
        double acc = 0.0;
        for (int t = 0; t < P.nmu; ++t) {
          long long vs;
          gptr ptr = cell_addr(st, B, P.mu_src[t], p3[0], p3[1], p3[2], vs);
          acc = fma(P.mu_a[t], ptr[v * vs], acc);
        }
        return acc;
      };
      // code word of interface i+1/2 = lower face of cell i+1
      auto code_at = [&](int i) -> unsigned long long {
        int p3[3] = {cc[0], cc[1], cc[2]};
        p3[D] = i + 1;
        if (i + 1 < nD) {
          const long long cell = ((long long)p3[2] * B.n[1] + p3[1]) * B.n[0] + p3[0];
          return *(__attribute__((address_space(1))) const unsigned long long*)(P.codes + D * P.code_plane +
                                                                               (B.coff + cell) * 8);
        }
        return *(__attribute__((address_space(1))) const unsigned long long*)(P.codes + D * P.code_plane +
                                                                             (P.code_faces + B.fco[D] + tr) * 8);
      };
      double lp[NV], lm[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) { lp[v] = 0.0; lm[v] = 0.0; }
      // interfaces i = m-3 .. m+2 that exist (-1 .. nD-1) and reach m
      for (int i = m - 3; i <= m + 2; ++i) {
        if (i < -1 || i > nD - 1) continue;
        const unsigned long long word = code_at(i);
        const int sp = m - (i - 2);   // position of m in the F+ stencil (cells i-2 .. i+2)
        const int sm = i + 3 - m;     // position of m in the F- stencil (cells i+3 .. i-1)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double lf = (mu_at(i + 1, v) - mu_at(i, v)) * idx_d;
          const int code = (int)((word >> (8 * v)) & 0xff);
          if (sp >= 0 && sp <= 4) lp[v] = fma(lf, piece_weight(P.recon, code & 15, sp), lp[v]);
          if (sm >= 0 && sm <= 4) lm[v] = fma(lf, piece_weight(P.recon, code >> 4, sm), lm[v]);
        }
      }
      // split adjoint and flux transpose at the ghost state (caller's values)
      int g3[3] = {cc[0], cc[1], cc[2]};
      g3[D] = m;
      long long vs;
      gptr ug = cell_addr(st, B, 0, g3[0], g3[1], g3[2], vs);
      double u[NV], lF[NV], nu[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        u[v] = ug[v * vs];
        nu[v] = 0.0;
      }
      PrimD w;
      prim<NDIM, MHD>(u, P.gamma, w);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        lF[v] = 0.5 * (lp[v] + lm[v]);
        const double dF = lp[v] - lm[v];
        nu[v] = fma(0.5 * c, dF, nu[v]);
        cp[D] = fma(0.5 * u[v], dF, cp[D]);
      }
      static_for<0, NDIM>([&](auto Dc) {
        constexpr int DD = decltype(Dc)::value;
        if (DD == D) flux_vjp<NDIM, MHD, DD>(u, w, P.gamma, lF, nu);
      });
      const long long g = B.gho[F.face] + q;
#pragma unroll
      for (int v = 0; v < NV; ++v) gadj[v * gplane + g] = fma(P.scale, nu[v], gadj[v * gplane + g]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) cp[d] = wave_sum(cp[d]);
  if ((tid & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) red[tid >> 6][d] = cp[d];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) cpart[3 * (long long)blockIdx.x + d] = (red[0][d] + red[1][d]) + (red[2][d] + red[3][d]);
  }
}

// Sum of the per-work-group c_max adjoints (fixed order: strided per
// thread, then a fixed butterfly per wave, then the 4 waves in order), then
// lam[argmax_d] += scale * lamc_d * d(|v_d| + c_f,d)/dU at the maximiser, for
// d in order.  Thread 0 issues the loads of the maximisers' keys, block
// entries, states and lambda values first, so they overlap the sum.
template <int NDIM, bool MHD>
__global__ void __launch_bounds__(256) k_vjp_cmax(StateTable st, int nblocks, const double* cpart, int nparts,
                                                  Control* ctl, double gamma, int in, int lam, double scale) {
  using E = Eq<NDIM, MHD>;
  constexpr int NV = E::NV;
  __shared__ double ws[4][3];
  const int tid = threadIdx.x;
  bool ok[NDIM];
  int bk[NDIM];
  long long ck[NDIM], wst[NDIM];
  double u[NDIM][NV], lv[NDIM][NV];
  gptr_w qd[NDIM];
  if (tid == 0) {
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      const long long key = ctl->arg[d];
      bk[d] = (int)(key >> 32);
      ck[d] = key & 0xffffffffll;
      // no cell had a finite speed (non-physical state): reported below, never indexed
      ok[d] = !(key < 0 || bk[d] < 0 || bk[d] >= nblocks) && ck[d] < st.blocks[bk[d]].cells;
      if (!ok[d]) continue;
      const BlockDev& B = st.blocks[bk[d]];
      const int i = (int)(ck[d] % B.n[0]), j = (int)((ck[d] / B.n[0]) % B.n[1]),
                k = (int)(ck[d] / ((long long)B.n[0] * B.n[1]));
      long long vs;
      gptr p = cell_addr(st, B, in, i, j, k, vs);
      qd[d] = (gptr_w)(cell_addr(st, B, lam, i, j, k, wst[d]));
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        u[d][v] = p[v * vs];
        lv[d][v] = qd[d][v * wst[d]];
      }
    }
  }
  double acc[3] = {0.0, 0.0, 0.0};
  for (int t = tid; t < nparts; t += 256)
#pragma unroll
    for (int d = 0; d < 3; ++d) acc[d] += cpart[3 * (long long)t + d];
#pragma unroll
  for (int d = 0; d < 3; ++d) acc[d] = wave_sum(acc[d]);
  if ((tid & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) ws[tid >> 6][d] = acc[d];
  }
  __syncthreads();
  if (tid != 0) return;
  double sd[3];
  for (int d = 0; d < 3; ++d) sd[d] = ((ws[0][d] + ws[1][d]) + ws[2][d]) + ws[3][d];
#pragma unroll
  for (int d = 0; d < NDIM; ++d) {
    if (!ok[d]) {
      atomicOr(&ctl->err, 1);
      break;
    }
    // the current lambda at the cell: updated by an earlier direction with
    // the same maximiser, else as loaded
    double cur[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) cur[v] = lv[d][v];
#pragma unroll
    for (int e = 0; e < d; ++e)
      if (bk[e] == bk[d] && ck[e] == ck[d])
#pragma unroll
        for (int v = 0; v < NV; ++v) cur[v] = lv[e][v];
    double lu[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) lu[v] = 0.0;
    speed_vjp<NDIM, MHD>(u[d], gamma, d, sd[d], lu);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      lv[d][v] = fma(scale, lu[v], cur[v]);
      qd[d][v * wst[d]] = lv[d][v];
    }
  }
  // the keys are consumed: ready for the next VJP's atomicMin
  for (int d = 0; d < 3; ++d) ctl->arg[d] = 0x7fffffffffffffffll;
}

// dst = sum_j a[j] * src[j] over the interiors (up to 6 terms; dst may be a
// source).

__global__ void __launch_bounds__(256) k_combine(CombineParams P) {
  const int tcells = P.tx * P.ty * P.tz;
  for (int t = blockIdx.x; t < P.ntiles; t += gridDim.x) {
    const Tile tl = P.tiles[t];
    const BlockDev& B = P.st.blocks[tl.block];
    for (int c = threadIdx.x; c < tcells; c += 256) {
      const int i = tl.o[0] + c % P.tx, j = tl.o[1] + (c / P.tx) % P.ty, k = tl.o[2] + c / (P.tx * P.ty);
      if (i >= B.n[0] || j >= B.n[1] || k >= B.n[2]) continue;
      long long vs[6], ws;
      gptr sp[6];
      for (int q = 0; q < P.n; ++q) sp[q] = cell_addr(P.st, B, P.src[q], i, j, k, vs[q]);
      gptr_w dp = (gptr_w)(cell_addr(P.st, B, P.dst, i, j, k, ws));
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
    gptr_w q = (gptr_w)(cell_addr(st, B, dst, i, j, k, ws));
    gptr src = (gptr)ptrs[b];
    for (int v = 0; v < nv; ++v) q[v * ws] = src[v * pstride + pidx];
  }
}

// Ghost entries: the boundary-data adjoint gadj (ghost cells of fixed faces,
// layout of BlockDev::gho) where gadj is given, else 0.
__global__ void __launch_bounds__(256) k_lam_export(StateTable st, double* const* ptrs, int nv, int src,
                                                    const double* gadj, long long gplane) {
  const int b = blockIdx.x;
  const BlockDev& B = st.blocks[b];
  const long long pstride = (long long)B.P[0] * B.P[1] * B.P[2];
  for (long long pc = threadIdx.x; pc < pstride; pc += 256) {
    const int pi = (int)(pc % B.P[0]), pj = (int)((pc / B.P[0]) % B.P[1]), pk = (int)(pc / ((long long)B.P[0] * B.P[1]));
    const int c3[3] = {pi - B.g[0], pj - B.g[1], pk - B.g[2]};
    int out = 0, od = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (c3[d] < 0 || c3[d] >= B.n[d]) { ++out; od = d; }
    gptr_w dst = (gptr_w)ptrs[b];
    if (out == 0) {
      long long vs;
      gptr p = cell_addr(st, B, src, c3[0], c3[1], c3[2], vs);
      for (int v = 0; v < nv; ++v) dst[v * pstride + pc] = p[v * vs];
      continue;
    }
    long long g = -1;
    if (gadj && out == 1) {
      const int side = c3[od] < 0 ? 0 : 1;
      const long long base = B.gho[2 * od + side];
      if (base >= 0) {
        const int layer = side == 0 ? -1 - c3[od] : c3[od] - B.n[od];
        const int e0 = od == 0 ? 1 : 0, e1 = od == 2 ? 1 : 2;
        const long long area = (long long)B.n[e0] * B.n[e1];
        g = base + layer * area + c3[e0] + (long long)B.n[e0] * c3[e1];
      }
    }
    for (int v = 0; v < nv; ++v) dst[v * pstride + pc] = g >= 0 ? gadj[v * gplane + g] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------

template <int NDIM, bool MHD, int TX, int TY, int TZ, int NT>
static void launch_vjp_t(const VjpParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_vjp<NDIM, MHD, TX, TY, TZ, NT>), dim3(grid), dim3(NT), 0, s, p);
}


template <int NDIM, bool MHD>
static void launch_cmax_term_t(StateTable st, int nblocks, const double* cpart, int ntiles, Control* ctl, double gamma,
                               int in, int lam, double scale, hipStream_t s) {
  hipLaunchKernelGGL((k_vjp_cmax<NDIM, MHD>), dim3(1), dim3(256), 0, s, st, nblocks, cpart, ntiles, ctl, gamma, in,
                     lam, scale);
}

template <int NDIM, bool MHD>
static void launch_ghost_t(const VjpParams& p, const FixedFace* faces, int nfaces, double* gadj, long long gplane,
                           double* cpart, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_vjp_ghost<NDIM, MHD>), dim3(grid), dim3(256), 0, s, p, faces, nfaces, gadj, gplane, cpart);
}

#define AMRVAC_VJP(ND, M, TX, TY, TZ, NT)                                                               \
  {ND, M, TX, TY, TZ, NT, (const void*)&k_vjp<ND, M, TX, TY, TZ, NT>, &launch_vjp_t<ND, M, TX, TY, TZ, NT>, \
   &launch_cmax_term_t<ND, M>, &launch_ghost_t<ND, M>}

// The VJP walks a tile list of its own shape (the recompute's list has the
// code-emitting stage kernel's shape).  3D ideal MHD takes 8x8x8 tiles: the
// halo rows of mu and the code words re-read per tile fall from 3 and 5.5 to
// 2.25 and 4.9 times the tile's own, at the same 2 waves per SIMD.
static const VjpVariant g_vjp[] = {
    AMRVAC_VJP(1, false, 64, 1, 1, 64),
    AMRVAC_VJP(1, true, 64, 1, 1, 64),
    AMRVAC_VJP(2, false, 16, 16, 1, 256),
    AMRVAC_VJP(2, true, 16, 16, 1, 256),
    AMRVAC_VJP(3, false, 8, 8, 4, 256),
    AMRVAC_VJP(3, true, 8, 8, 8, 512),
};

const VjpVariant* vjp_variant(int ndim, int mhd) {
  for (const VjpVariant& v : g_vjp)
    if (v.ndim == ndim && v.mhd == mhd) return &v;
  return nullptr;
}


void launch_combine(const CombineParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(grid), dim3(256), 0, s, p);
}

void launch_lam_import(StateTable st, double* const* ptrs, int nv, int dst, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_lam_import, dim3(nblocks), dim3(256), 0, s, st, ptrs, nv, dst);
}

void launch_lam_export(StateTable st, double* const* ptrs, int nv, int src, int nblocks, const double* gadj,
                       long long gplane, hipStream_t s) {
  hipLaunchKernelGGL(k_lam_export, dim3(nblocks), dim3(256), 0, s, st, ptrs, nv, src, gadj, gplane);
}

}  // namespace amrvac
