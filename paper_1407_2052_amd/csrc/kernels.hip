// gfx950 (MI355X) FP64 kernels of the conservative finite-difference scheme
// of Porth et al. (2014), Sect. 2:
//   * k_stage: one fused Shu-Osher stage (Sect. 2.3) on tiles of blocks:
//     halo load -> primitive recovery -> physical flux -> global
//     Lax-Friedrichs split (Sect. 2.2) -> MP5 or LIM03 of F+ (left-biased)
//     and F- (right-biased) -> interface flux -> conservative difference
//     (Sect. 2.1, eq. fdcons) -> stage combination -> |v_d| + c_f,d of the
//     new state for the next stage's c_max.  Template flags select LIM03,
//     GLM-MHD (Sect. 4.2, glm3) and Hall MHD (Sect. 4.4), and the
//     code-emitting form of the adjoint's recompute;
//   * k_cmax: c_max of a state (Sect. 2.2);
//   * k_step_begin: dt from c_max (multi-D form of the Sect. 4.4 bound),
//     t accumulation, the GLM decay factor and c_max slot resets, so a
//     whole step runs without a host round trip;
//   * k_current: the cell-centred current of Hall MHD (Sect. 4.4);
//   * k_divb, k_sum_fixed: the div B monitor of Sect. 4.5.1.
//
// Work decomposition.  A tile is a TX x TY x TZ box of one block's interior;
// one work-group owns one tile at a time and loops over tiles (persistent
// grid).  Per direction d and per group of variables the work-group
//   A) computes F+ and F- for the tile extended by 3 cells along d (2 for
//      LIM03; halo cells come from the neighbour's interior or the fixed
//      ghost layers) into LDS,
//   B) evaluates R(F+) + R(F-) for every (interface, variable) of the tile
//      (T_d + 1 interfaces per pencil), per interface or in runs of up to 5
//      interfaces per pencil, into registers, then LDS,
//   C) accumulates -(Fhat_{i+1/2} - Fhat_{i-1/2}) / dx_d into per-thread
//      register accumulators of the cells it owns.
// In the run forms the interface fluxes of B go beside the split fluxes of A
// in LDS wherever both fit (the array is padded for that while it keeps the
// resident work-groups per CU), which drops the barrier before they are
// stored and, when the next direction's split fluxes also stay clear of
// them, the barrier after C.
// The stage update reads its sources once per cell and writes the result.
// The owned-cell (CORE) forms load the tile's own cells once per tile into
// registers; phase A of each direction then loads only the halo planes of the
// extended box along d, and the stage update takes the source that equals
// the stage input from the same registers.  The traffic beyond the
// algorithmic state passes is the re-reading of those halo planes, which L2
// serves only in part (the more tiles are in flight per XCD, the less).
//
// Floating point: automatic FMA contraction is off for this file (the build
// passes -ffp-contract=off) and every fused multiply-add is written
// explicitly, so the arithmetic is fixed by the source: every tile shape,
// both execution forms and the adjoint's forward recompute produce bitwise
// identical results.
//
// Accumulation order of L matches the definition: L = 0; for d: L -= diff_d
// / dx_d (as a product with 1/dx_d).  MP5 is evaluated in its median form
// median(fL, fmin, fmax); with eps = 0 the early exit of the published
// algorithm returns the same value (fL lies inside both bounds whenever the
// early-exit test holds).
#include "device_math.h"

namespace amrvac {

// ---------------------------------------------------------------------------
// Fused stage kernel.
// ---------------------------------------------------------------------------
// LDS doubles of direction D in a run form with the interface fluxes (and
// code bytes) beside the split fluxes of the extended box.
template <class S, int VPG, int XP, bool CODES>
constexpr int side_by_side(int D) {
  return 2 * VPG * (D == 0 ? XP * S::T(1) * S::T(2) : S::NEXT(D)) + (VPG + (CODES ? 1 : 0)) * S::NIFC(D);
}

template <int NDIM, bool MHD, int TX, int TY, int TZ, int NT, int NGRP, int WPE, bool EMIT = false,
          bool RUNS = false, bool LIM = false, bool GLM = false, bool HALL = false, bool CORE = false>
__global__ void __launch_bounds__(NT, WPE) k_stage(StageParams P) {
  static_assert(!HALL || (MHD && !GLM), "Hall terms are built for ideal MHD");
  // halo of the extended box: MP5 reaches 3 cells, LIM03 2
  constexpr int HG = LIM ? 2 : NG;
  using E = Eq<NDIM, MHD, GLM>;
  using S = TileShape<TX, TY, TZ, HG>;
  constexpr int NV = E::NV;
  constexpr int VPG = (NV + NGRP - 1) / NGRP;
  constexpr int TC = S::TC;
  constexpr int CPT = (TC + NT - 1) / NT;
  // with RUNS the x rows of the extended box get an odd LDS stride
  constexpr int XP = RUNS ? ((TX + 2 * HG) | 1) : TX + 2 * HG;
  constexpr int EXT = cmax_i<cmax_i<XP * TY * TZ, NDIM >= 2 ? S::NEXT(1) : 0>::v,
                             NDIM >= 3 ? S::NEXT(2) : 0>::v;
  constexpr int IFC = cmax_i<cmax_i<S::NIFC(0), NDIM >= 2 ? S::NIFC(1) : 0>::v,
                             NDIM >= 3 ? S::NIFC(2) : 0>::v;
  // code-emitting run forms with one variable group stage the piece codes of
  // a direction in LDS after the interface fluxes (8 bytes per interface,
  // byte v for variable v) and store them as one 8-byte word per cell face
  constexpr bool CODE_LDS = EMIT && RUNS && NGRP == 1;
  static_assert(!EMIT || CODE_LDS, "the code-emitting forms are run forms with one variable group");
  static_assert(!CODE_LDS || NV <= 8, "8 code bytes per interface");
  constexpr int LDS_BASE = cmax_i<2 * VPG * EXT, VPG * IFC + (CODE_LDS ? IFC : 0)>::v;
  // Run forms: the interface fluxes (and codes) of a direction go to the top
  // of the array when they fit beside that direction's split fluxes; then the
  // barrier between the reconstructions and their store is not needed, nor
  // the one after phase C when the next split fluxes stay clear of them too.
  // The array grows to fit every direction that can be placed so without
  // fewer resident work-groups per CU (160 KB of LDS per CU) than the launch
  // bounds aim at and the unpadded array allows.
  constexpr int WG_BASE = 20480 / LDS_BASE;
  constexpr int WG_AIM = cmax_i<WPE * 4 / (NT / 64), 1>::v;
  constexpr int LDS_LIMIT = 20480 / (WG_BASE < WG_AIM ? WG_BASE : WG_AIM);
  constexpr int SB0 = side_by_side<S, VPG, XP, CODE_LDS>(0);
  constexpr int SB1 = NDIM >= 2 ? side_by_side<S, VPG, XP, CODE_LDS>(1) : 0;
  constexpr int SB2 = NDIM >= 3 ? side_by_side<S, VPG, XP, CODE_LDS>(2) : 0;
  constexpr int PAD = !(RUNS && NGRP == 1) ? 0
                      : cmax_i<cmax_i<SB0 <= LDS_LIMIT ? SB0 : 0, SB1 <= LDS_LIMIT ? SB1 : 0>::v,
                               SB2 <= LDS_LIMIT ? SB2 : 0>::v;
  constexpr int LDS_N = cmax_i<LDS_BASE, PAD>::v;
  __shared__ double lds[LDS_N];
  // the closing c_max reduction reuses the start of lds: every wave has
  // passed the barrier that ends the last phase C before any writes it
  static_assert(LDS_N >= 3 * (NT / 64), "lds too small for the c_max reduction");
  double (*red)[3] = reinterpret_cast<double (*)[3]>(lds);

  const int tid = threadIdx.x;
  const StateTable& st = P.st;
  Control* ctl = P.ctl;
  const double gamma = P.gamma;

  double cin[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) cin[d] = __longlong_as_double((long long)ctl->cm[P.cm_in][d]);
  if constexpr (GLM) {
    // the cleaning speed c_h = max_d c_max,d serves every direction
    double ch = cin[0];
#pragma unroll
    for (int d = 1; d < NDIM; ++d) ch = fmax(ch, cin[d]);
#pragma unroll
    for (int d = 0; d < NDIM; ++d) cin[d] = ch;
  }
  const double dt = (P.mode == 0) ? ctl->dt : 0.0;
  const double psi_decay = (GLM && P.decay_psi) ? ctl->psi_decay : 1.0;
  const double dtb = dt * P.b;
  const double dtsb = dt * P.sb;
  if (EMIT && P.cm_hist && blockIdx.x == 0 && tid == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) P.cm_hist[d] = __longlong_as_double((long long)ctl->cm[P.cm_in][d]);
  }
  if (P.cm_reset >= 0 && blockIdx.x == 0 && tid == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) ctl->cm[P.cm_reset][d] = 0ull;
  }

  double run[3] = {0.0, 0.0, 0.0};
  bool ok_all = true;

  const TileSchedule sched(P.ntiles);
  for (int t = sched.t; t < sched.end; t += sched.step) {
    const Tile tl = P.tiles[P.tile_begin + t];
    const BlockDev& B = st.blocks[tl.block];
    int tend[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int rem = B.n[d] - tl.o[d];
      tend[d] = rem < S::T(d) ? rem : S::T(d);
    }

    double L[CPT][NV];
#pragma unroll
    for (int r = 0; r < CPT; ++r)
#pragma unroll
      for (int v = 0; v < NV; ++v) L[r][v] = 0.0;

    // CORE: the owned cells' state of buffer `in`, read once per tile; every
    // direction's phase A then takes the owned cells from registers and loads
    // only the halo planes, and the stage update takes the source equal to
    // `in` from registers too.
    double uc[CORE ? CPT : 1][NV];
    if constexpr (CORE) {
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int cidx = tid + r * NT;
        const int a0 = cidx % TX, a1 = (cidx / TX) % TY, a2 = cidx / (TX * TY);
        if (cidx < TC && a0 < tend[0] && a1 < tend[1] && a2 < tend[2]) {
          long long vs;
          gptr p = cell_addr(st, B, P.in, tl.o[0] + a0, tl.o[1] + a1, tl.o[2] + a2, vs);
#pragma unroll
          for (int v = 0; v < NV; ++v) uc[r][v] = p[v * vs];
        }
      }
    }

    static_for<0, NDIM>([&](auto Dc) {
      constexpr int D = decltype(Dc)::value;
      constexpr int E0 = S::E(D, 0), E1 = S::E(D, 1);
      constexpr int E0P = (D == 0) ? XP : E0;            // LDS row stride of the extended box
      constexpr int NEXT_D = S::NEXT(D);
      constexpr int NEXTP = E0P * E1 * S::E(D, 2);       // LDS size of one variable's box
      constexpr int NIFC_D = S::NIFC(D);
      constexpr int NITEM = VPG * NIFC_D;
      constexpr int IPT = (NITEM + NT - 1) / NT;
      constexpr int I0 = S::I(D, 0), I1 = S::I(D, 1);
      constexpr int SD = (D == 0) ? 1 : (D == 1) ? E0P : E0P * E1;
      // interface fluxes at lds[RB ..]: beside the split fluxes (DISJ) or over them
      constexpr int RES_SPAN = VPG * NIFC_D + (CODE_LDS ? NIFC_D : 0);
      constexpr bool DISJ = RUNS && NGRP == 1 && 2 * VPG * NEXTP + RES_SPAN <= LDS_N;
      constexpr int RB = DISJ ? LDS_N - RES_SPAN : 0;
      // what is written to LDS after phase C: the next direction's split
      // fluxes, or the next tile's first ones and the closing reduction
      constexpr int DN = D + 1 < NDIM ? D + 1 : 0;
      constexpr int NEXT_SPAN = cmax_i<2 * VPG * (DN == 0 ? XP : S::E(DN, 0)) * S::E(DN, 1) * S::E(DN, 2),
                                       3 * (NT / 64)>::v;
      constexpr bool SKIP_C_BARRIER = DISJ && NEXT_SPAN <= RB;
      const double c = cin[D];
      const double idx_d = B.inv_dx[D];
      // LIM03's asymptotic-region scale 1 / (r dx_d)^2
      const double kr = (idx_d * (1.0 / LIM03_RADIUS)) * (idx_d * (1.0 / LIM03_RADIUS));

      static_for<0, NGRP>([&](auto Gc) {
        constexpr int G = decltype(Gc)::value;
        // A) split fluxes of the extended tile -> LDS.  split_to_lds: state u
        // of the cell at extended-box position a (block coordinates cc).
        auto split_to_lds = [&](const double* u, const int* a, const int* cc) {
          PrimD w;
          ok_all = prim<NDIM, MHD>(u, gamma, w) && ok_all;
          double F[NV];
          phys_flux<NDIM, MHD, D>(u, w, F);
          if constexpr (GLM) {
            F[5 + D] += u[8];             // psi on the flux of B_D
            F[8] = (c * c) * u[5 + D];    // c_h^2 B_D
          }
          if constexpr (HALL) {
            // (eta_h/rho)(B_D J - J_D B) on B, (eta_h/rho)((J.B) B_D - B^2 J_D) on E
            double Jc[3];
#pragma unroll
            for (int v = 0; v < 3; ++v) Jc[v] = load_plane<D>(st, P.J, P.jplane, v, tl.block, cc[0], cc[1], cc[2]);
            const double h = P.eta_h / w.rho;
            const double jb = Jc[0] * w.B[0] + Jc[1] * w.B[1] + Jc[2] * w.B[2];
            const double bb = w.B[0] * w.B[0] + w.B[1] * w.B[1] + w.B[2] * w.B[2];
            const double Bd = w.B[D];
#pragma unroll
            for (int k = 0; k < 3; ++k) F[5 + k] = F[5 + k] + h * (Bd * Jc[k] - Jc[D] * w.B[k]);
            F[4] = F[4] + h * (jb * Bd - bb * Jc[D]);
          }
          const int el = a[0] + E0P * (a[1] + E1 * a[2]);
#pragma unroll
          for (int vg = 0; vg < VPG; ++vg) {
            const int v = G * VPG + vg;
            if (v < NV) {
              lds[vg * NEXTP + el] = 0.5 * fma(c, u[v], F[v]);
              lds[(VPG + vg) * NEXTP + el] = 0.5 * fma(-c, u[v], F[v]);
            }
          }
        };
        if constexpr (CORE) {
          // the 2 HG halo planes along D from memory (plane p < HG is
          // extended-box row p, plane p >= HG row tend_D + p): every load of
          // this thread is issued first, and the owned cells, which come from
          // registers, are converted while the loads are in flight
          constexpr int H0 = D == 0 ? 2 * HG : TX, H1 = D == 1 ? 2 * HG : TY, H2 = D == 2 ? 2 * HG : TZ;
          constexpr int NH = H0 * H1 * H2;
          constexpr int HPT = (NH + NT - 1) / NT;
          double hu[HPT][NV];
          int ha[HPT][3];
          bool hok[HPT];
#pragma unroll
          for (int r = 0; r < HPT; ++r) {
            const int h = tid + r * NT;
            ha[r][0] = h % H0;
            ha[r][1] = (h / H0) % H1;
            ha[r][2] = h / (H0 * H1);
            bool valid = h < NH;
#pragma unroll
            for (int d = 0; d < 3; ++d)
              if (d != D) valid = valid && (ha[r][d] < tend[d]);
            if (ha[r][D] >= HG) ha[r][D] += tend[D];
            hok[r] = valid;
            if (valid) {
              int cc[3];
#pragma unroll
              for (int d = 0; d < 3; ++d) cc[d] = tl.o[d] + ha[r][d] - (d == D ? HG : 0);
              load_cell<NV, D>(st, tl.block, P.in, cc[0], cc[1], cc[2], hu[r]);
            }
          }
          // owned cells from registers
#pragma unroll
          for (int r = 0; r < CPT; ++r) {
            const int cidx = tid + r * NT;
            int a[3] = {cidx % TX, (cidx / TX) % TY, cidx / (TX * TY)};
            if (cidx < TC && a[0] < tend[0] && a[1] < tend[1] && a[2] < tend[2]) {
              const int cc[3] = {tl.o[0] + a[0], tl.o[1] + a[1], tl.o[2] + a[2]};
              a[D] += HG;
              split_to_lds(uc[r], a, cc);
            }
          }
#pragma unroll
          for (int r = 0; r < HPT; ++r) {
            if (!hok[r]) continue;
            int cc[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) cc[d] = tl.o[d] + ha[r][d] - (d == D ? HG : 0);
            split_to_lds(hu[r], ha[r], cc);
          }
        } else {
          for (int e = tid; e < NEXT_D; e += NT) {
            int a[3];
            a[0] = e % E0;
            a[1] = (e / E0) % E1;
            a[2] = e / (E0 * E1);
            bool valid = true;
            int cc[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              if (d == D) {
                valid = valid && (a[d] < tend[d] + 2 * HG);
                cc[d] = tl.o[d] + a[d] - HG;
              } else {
                valid = valid && (a[d] < tend[d]);
                cc[d] = tl.o[d] + a[d];
              }
            }
            if (valid) {
              double u[NV];
              load_cell<NV, D>(st, tl.block, P.in, cc[0], cc[1], cc[2], u);
              split_to_lds(u, a, cc);
            }
          }
        }
        __syncthreads();
        // B) interface fluxes for every (variable, interface)
        if constexpr (RUNS) {
          // one item per (variable, pencil, run of up to 5 interfaces): the
          // run reads every split flux of its window once and, for MP5,
          // shares curvatures and curvature limiters between its
          // interfaces.  The last run of a pencil is shifted back to end at
          // the pencil's last interface.
          constexpr int NIF = S::T(D) + 1;
          constexpr int RUN = NIF < 5 ? NIF : 5;
          constexpr int NRUN = (NIF + RUN - 1) / RUN;
          constexpr int NPEN = NIFC_D / NIF;
          constexpr int NIT = VPG * NPEN * NRUN;
          constexpr int IPR = (NIT + NT - 1) / NT;
          double res[IPR][RUN];
          unsigned char cbyte[CODE_LDS ? IPR : 1][RUN];
#pragma unroll
          for (int r = 0; r < IPR; ++r) {
            const int w = tid + r * NT;
#pragma unroll
            for (int kk = 0; kk < RUN; ++kk) res[r][kk] = 0.0;
            if constexpr (CODE_LDS) {
#pragma unroll
              for (int kk = 0; kk < RUN; ++kk) cbyte[r][kk] = 0;
            }
            if (w >= NIT) continue;
            const int pen = w % NPEN;
            const int run = (w / NPEN) % NRUN;
            const int vg = w / (NPEN * NRUN);
            const int k0 = run * RUN < NIF - RUN ? run * RUN : NIF - RUN;
            int a[3];
            if constexpr (D == 0) { a[0] = k0; a[1] = pen % TY; a[2] = pen / TY; }
            if constexpr (D == 1) { a[0] = pen % TX; a[1] = k0; a[2] = pen / TX; }
            if constexpr (D == 2) { a[0] = pen % TX; a[1] = pen / TX; a[2] = k0; }
            bool valid = (G * VPG + vg) < NV;
#pragma unroll
            for (int d = 0; d < 3; ++d)
              if (d != D) valid = valid && (a[d] < tend[d]);
            if (!valid) continue;
            // interface a_D lies between cells a_D - 1 and a_D; its F+
            // stencil is ext a_D .. a_D + 2 HG - 2, its F- stencil ext
            // a_D + 2 HG - 1 .. a_D + 1 (mirrored).  fp and fm hold the run's
            // windows, so that interface kk of the run reconstructs F+ from
            // fp[kk ..] and F- from fm[RUN - 1 - kk ..].
            constexpr int W = RUN + 2 * HG - 2;
            const int eb = a[0] + E0P * (a[1] + E1 * a[2]);
            // one window at a time (F+, then F-) keeps fewer registers live;
            // res = R(F+) + R(F-) in that operand order either way
            int cp[RUN], cm[RUN];
            {
              double fw[W], o[RUN];
#pragma unroll
              for (int m = 0; m < W; ++m) fw[m] = lds[vg * NEXTP + eb + m * SD];
              if constexpr (LIM) {
#pragma unroll
                for (int kk = 0; kk < RUN; ++kk) o[kk] = lim03_eval<EMIT>(fw[kk], fw[kk + 1], fw[kk + 2], kr, cp[kk]);
              } else {
                mp5_run<RUN, EMIT>(fw, o, cp);
              }
#pragma unroll
              for (int kk = 0; kk < RUN; ++kk) res[r][kk] = o[kk];
            }
            {
              double fw[W], o[RUN];
#pragma unroll
              for (int m = 0; m < W; ++m) fw[m] = lds[(VPG + vg) * NEXTP + eb + (W - m) * SD];
              if constexpr (LIM) {
#pragma unroll
                for (int kk = 0; kk < RUN; ++kk) o[kk] = lim03_eval<EMIT>(fw[kk], fw[kk + 1], fw[kk + 2], kr, cm[kk]);
              } else {
                mp5_run<RUN, EMIT>(fw, o, cm);
              }
#pragma unroll
              for (int kk = 0; kk < RUN; ++kk) res[r][kk] = res[r][kk] + o[RUN - 1 - kk];
            }
            if constexpr (CODE_LDS) {
#pragma unroll
              for (int kk = 0; kk < RUN; ++kk) cbyte[r][kk] = (unsigned char)(cp[kk] | (cm[RUN - 1 - kk] << 4));
            }
          }
          if constexpr (!DISJ) __syncthreads();
#pragma unroll
          for (int r = 0; r < IPR; ++r) {
            const int w = tid + r * NT;
            if (w >= NIT) continue;
            const int pen = w % NPEN;
            const int run = (w / NPEN) % NRUN;
            const int vg = w / (NPEN * NRUN);
            const int k0 = run * RUN < NIF - RUN ? run * RUN : NIF - RUN;
            int a[3];
            if constexpr (D == 0) { a[0] = k0; a[1] = pen % TY; a[2] = pen / TY; }
            if constexpr (D == 1) { a[0] = pen % TX; a[1] = k0; a[2] = pen / TX; }
            if constexpr (D == 2) { a[0] = pen % TX; a[1] = pen / TX; a[2] = k0; }
            const int q0 = a[0] + I0 * (a[1] + I1 * a[2]);
            constexpr int SI = S::SI(D);
#pragma unroll
            for (int kk = 0; kk < RUN; ++kk) lds[RB + vg * NIFC_D + q0 + kk * SI] = res[r][kk];
            if constexpr (CODE_LDS) {
              if ((G * VPG + vg) < NV) {
                unsigned char* lc = reinterpret_cast<unsigned char*>(lds + RB + VPG * NIFC_D);
#pragma unroll
                for (int kk = 0; kk < RUN; ++kk) lc[(q0 + kk * SI) * 8 + vg] = cbyte[r][kk];
              }
            }
          }
          __syncthreads();
          if constexpr (CODE_LDS) {
            // one 8-byte word per owned cell: the codes of the interface on
            // its lower face (unused bytes of a hydro word stay unspecified)
            const unsigned long long* lc = reinterpret_cast<const unsigned long long*>(lds + RB + VPG * NIFC_D);
#pragma unroll
            for (int r = 0; r < CPT; ++r) {
              const int cidx = tid + r * NT;
              if (cidx >= TC) continue;
              const int a0 = cidx % TX, a1 = (cidx / TX) % TY, a2 = cidx / (TX * TY);
              if (!(a0 < tend[0] && a1 < tend[1] && a2 < tend[2])) continue;
              const long long cell = ((long long)(tl.o[2] + a2) * B.n[1] + (tl.o[1] + a1)) * B.n[0] + (tl.o[0] + a0);
              __attribute__((address_space(1))) unsigned long long* cw =
                  (__attribute__((address_space(1))) unsigned long long*)(P.codes + D * P.code_plane);
              const int il = a0 + I0 * (a1 + I1 * a2);
              cw[B.coff + cell] = lc[il];
              // the last cell of a fixed upper face: also the interface on its
              // upper face, in the words after the interior cells
              const int ac[3] = {tl.o[0] + a0, tl.o[1] + a1, tl.o[2] + a2};
              if (B.fco[D] >= 0 && ac[D] == B.n[D] - 1) {
                const long long tr = D == 0 ? (long long)ac[1] + (long long)B.n[1] * ac[2]
                                   : D == 1 ? (long long)ac[0] + (long long)B.n[0] * ac[2]
                                            : (long long)ac[0] + (long long)B.n[0] * ac[1];
                cw[P.code_faces + B.fco[D] + tr] = lc[il + S::SI(D)];
              }
            }
          }
        } else {
          double res[IPT];
#pragma unroll
          for (int r = 0; r < IPT; ++r) {
            const int w = tid + r * NT;
            res[r] = 0.0;
            if (w < NITEM) {
              const int vg = w / NIFC_D;
              const int q = w - vg * NIFC_D;
              int a[3];
              a[0] = q % I0;
              a[1] = (q / I0) % I1;
              a[2] = q / (I0 * I1);
              bool valid = (G * VPG + vg) < NV;
#pragma unroll
              for (int d = 0; d < 3; ++d) valid = valid && (a[d] < tend[d] + (d == D ? 1 : 0));
              if (valid) {
                // interface between cells a_D - 1 and a_D (tile coordinates);
                // stencil cells a_D - HG .. a_D + HG - 1 are ext indices
                // a_D .. a_D + 2 HG - 1
                int eb = 0;
                {
                  int ea[3] = {a[0], a[1], a[2]};
                  eb = ea[0] + E0P * (ea[1] + E1 * ea[2]);
                }
                const double* fp = &lds[vg * NEXTP + eb];
                const double* fm = &lds[(VPG + vg) * NEXTP + eb];
                if constexpr (LIM) {
                  // F+ from cells a_D - 2 .. a_D, F- mirrored from a_D + 1 .. a_D - 1
                  res[r] = lim03(fp[0], fp[SD], fp[2 * SD], kr) + lim03(fm[3 * SD], fm[2 * SD], fm[SD], kr);
                } else {
                  res[r] = mp5(fp[0], fp[SD], fp[2 * SD], fp[3 * SD], fp[4 * SD]) +
                           mp5(fm[5 * SD], fm[4 * SD], fm[3 * SD], fm[2 * SD], fm[SD]);
                }
              }
            }
          }
          __syncthreads();
#pragma unroll
          for (int r = 0; r < IPT; ++r) {
            const int w = tid + r * NT;
            if (w < NITEM) lds[w] = res[r];
          }
          __syncthreads();
        }
        // C) conservative difference into the owned cells
#pragma unroll
        for (int r = 0; r < CPT; ++r) {
          const int cidx = tid + r * NT;
          if (cidx < TC) {
            int a[3];
            a[0] = cidx % TX;
            a[1] = (cidx / TX) % TY;
            a[2] = cidx / (TX * TY);
            if (a[0] < tend[0] && a[1] < tend[1] && a[2] < tend[2]) {
              const int il = a[0] + I0 * (a[1] + I1 * a[2]);
              constexpr int SI = S::SI(D);
#pragma unroll
              for (int vg = 0; vg < VPG; ++vg) {
                const int v = G * VPG + vg;
                if (v < NV) {
                  const double diff = lds[RB + vg * NIFC_D + il + SI] - lds[RB + vg * NIFC_D + il];
                  L[r][v] = fma(-diff, idx_d, L[r][v]);
                }
              }
            }
          }
        }
        if constexpr (!SKIP_C_BARRIER) __syncthreads();
      });
    });

    // Stage update (or right-hand side output) and next-stage speeds.
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      const int cidx = tid + r * NT;
      if (cidx >= TC) continue;
      int a[3];
      a[0] = cidx % TX;
      a[1] = (cidx / TX) % TY;
      a[2] = cidx / (TX * TY);
      if (!(a[0] < tend[0] && a[1] < tend[1] && a[2] < tend[2])) continue;
      const int i = tl.o[0] + a[0], j = tl.o[1] + a[1], k = tl.o[2] + a[2];
      if (P.mode == 1) {
        gptr_w out = (gptr_w)(P.rhs_out[tl.block] + (((long long)k * B.n[1] + j) * B.n[0] + i));
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v * B.cells] = L[r][v];
        continue;
      }
      double un[NV];
      if constexpr (CORE) {
        // the same sum, source by source; the source equal to `in` from
        // registers
        double acc[NV];
#pragma unroll
        for (int q = 0; q < MAX_SRC; ++q) {
          if (q >= P.nsrc) continue;
          if (P.src[q] == P.in) {
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = q == 0 ? P.a[0] * uc[CORE ? r : 0][v] : fma(P.a[q], uc[CORE ? r : 0][v], acc[v]);
          } else {
            long long vs;
            gptr sp = cell_addr(st, B, opaque_uniform(P.src[q]), i, j, k, vs);
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = q == 0 ? P.a[0] * sp[v * vs] : fma(P.a[q], sp[v * vs], acc[v]);
          }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) un[v] = fma(dtb, L[r][v], acc[v]);
      } else {
        long long vs[MAX_SRC];
        gptr sp[MAX_SRC];
#pragma unroll
        for (int q = 0; q < MAX_SRC; ++q)
          if (q < P.nsrc) sp[q] = cell_addr(st, B, opaque_uniform(P.src[q]), i, j, k, vs[q]);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double acc = P.a[0] * sp[0][v * vs[0]];
#pragma unroll
          for (int q = 1; q < MAX_SRC; ++q)
            if (q < P.nsrc) acc = fma(P.a[q], sp[q][v * vs[q]], acc);
          un[v] = fma(dtb, L[r][v], acc);
        }
      }
      {
        if constexpr (GLM) {
          if (P.decay_psi) un[8] = un[8] * psi_decay;   // operator-split decay of psi
        }
      }
      if (P.sdst >= 0) {
        long long vs[MAX_SRC];
        gptr sp[MAX_SRC];
        long long ws;
        gptr_w sd = cell_addr_w(st, B, opaque_uniform(P.sdst), i, j, k, ws);
        if constexpr (CORE) {
          double acc[NV];
#pragma unroll
          for (int q = 0; q < MAX_SRC; ++q) {
            if (q >= P.snsrc) continue;
            if (P.ssrc[q] == P.in) {
#pragma unroll
              for (int v = 0; v < NV; ++v)
                acc[v] = q == 0 ? P.sa[0] * uc[CORE ? r : 0][v] : fma(P.sa[q], uc[CORE ? r : 0][v], acc[v]);
            } else {
              long long vq;
              gptr spq = cell_addr(st, B, opaque_uniform(P.ssrc[q]), i, j, k, vq);
#pragma unroll
              for (int v = 0; v < NV; ++v) acc[v] = q == 0 ? P.sa[0] * spq[v * vq] : fma(P.sa[q], spq[v * vq], acc[v]);
            }
          }
#pragma unroll
          for (int v = 0; v < NV; ++v) sd[v * ws] = fma(dtsb, L[r][v], acc[v]);
        } else {
#pragma unroll
          for (int q = 0; q < MAX_SRC; ++q)
            if (q < P.snsrc) sp[q] = cell_addr(st, B, opaque_uniform(P.ssrc[q]), i, j, k, vs[q]);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            double acc = P.sa[0] * sp[0][v * vs[0]];
#pragma unroll
            for (int q = 1; q < MAX_SRC; ++q)
              if (q < P.snsrc) acc = fma(P.sa[q], sp[q][v * vs[q]], acc);
            sd[v * ws] = fma(dtsb, L[r][v], acc);
          }
        }
      }
      {
        long long ws;
        gptr_w dp = cell_addr_w(st, B, opaque_uniform(P.dst), i, j, k, ws);
#pragma unroll
        for (int v = 0; v < NV; ++v) dp[v * ws] = un[v];
      }
      if (P.cm_out >= 0) {
        PrimD w;
        ok_all = prim<NDIM, MHD>(un, gamma, w) && ok_all;
        if constexpr (HALL) {
          double km = B.inv_dx[0];
#pragma unroll
          for (int d = 1; d < NDIM; ++d) km = fmax(km, B.inv_dx[d]);
          const double wh = whistler_speed(w, P.eta_h, M_PI * km);
#pragma unroll
          for (int d = 0; d < NDIM; ++d) run[d] = fmax(run[d], fabs(w.v[d]) + fmax(fast_speed<MHD>(w, d, gamma), wh));
        } else {
#pragma unroll
          for (int d = 0; d < NDIM; ++d) run[d] = fmax(run[d], fabs(w.v[d]) + fast_speed<MHD>(w, d, gamma));
        }
      }
    }
  }

  // Fold the work-group maxima into the next stage's c_max slot.
  if (P.cm_out >= 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) run[d] = wave_max(run[d]);
    const int wv = tid >> 6, ln = tid & 63;
    if (ln == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) red[wv][d] = run[d];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
      for (int d = 0; d < NDIM; ++d) {
        double m = red[0][d];
        for (int q = 1; q < NT / 64; ++q) m = fmax(m, red[q][d]);
        atomicMax(&ctl->cm[P.cm_out][d], (unsigned long long)__double_as_longlong(m));
      }
    }
  }
  if (!ok_all) atomicOr(&ctl->err, 1);
}

// ---------------------------------------------------------------------------
// c_max of a state (interior cells of every block).
// ---------------------------------------------------------------------------
template <int NDIM, bool MHD>
__global__ void __launch_bounds__(256) k_cmax(CmaxParams P) {
  using E = Eq<NDIM, MHD>;
  constexpr int NV = E::NV;
  __shared__ double red[4][3];
  const int tid = threadIdx.x;
  double run[3] = {0.0, 0.0, 0.0};
  bool ok_all = true;
  const int tcells = P.tx * P.ty * P.tz;
  for (int t = blockIdx.x; t < P.ntiles; t += gridDim.x) {
    const Tile tl = P.tiles[t];
    const BlockDev& B = P.st.blocks[tl.block];
    for (int c = tid; c < tcells; c += 256) {
      const int i = tl.o[0] + c % P.tx;
      const int j = tl.o[1] + (c / P.tx) % P.ty;
      const int k = tl.o[2] + c / (P.tx * P.ty);
      if (i >= B.n[0] || j >= B.n[1] || k >= B.n[2]) continue;
      long long vs;
      gptr p = cell_addr(P.st, B, P.in, i, j, k, vs);
      double u[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = p[v * vs];
      PrimD w;
      ok_all = prim<NDIM, MHD>(u, P.gamma, w) && ok_all;
      double wh = 0.0;   // Hall MHD: fast whistler at k_max of the block
      if (MHD && P.eta_h != 0.0) {
        double km = B.inv_dx[0];
        for (int d = 1; d < NDIM; ++d) km = fmax(km, B.inv_dx[d]);
        wh = whistler_speed(w, P.eta_h, M_PI * km);
      }
#pragma unroll
      for (int d = 0; d < NDIM; ++d) run[d] = fmax(run[d], fabs(w.v[d]) + fmax(fast_speed<MHD>(w, d, P.gamma), wh));
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) run[d] = wave_max(run[d]);
  if ((tid & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) red[tid >> 6][d] = run[d];
  }
  __syncthreads();
  if (tid == 0) {
    for (int d = 0; d < NDIM; ++d) {
      double m = fmax(fmax(red[0][d], red[1][d]), fmax(red[2][d], red[3][d]));
      atomicMax(&P.ctl->cm[P.slot][d], (unsigned long long)__double_as_longlong(m));
    }
  }
  if (!ok_all) atomicOr(&P.ctl->err, 1);
}

// dt from c_max (or the fixed step), t += dt, and clearing of the c_max
// slots the coming stages accumulate into.  One thread.
__global__ void k_step_begin(Control* ctl, const double* dxtab, int ndim, int glm, int clear_lo,
                             int clear_hi) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double cm[3];
  for (int d = 0; d < 3; ++d) cm[d] = __longlong_as_double((long long)ctl->cm[0][d]);
  double ch = cm[0];
  if (glm) {   // every direction moves at the cleaning speed c_h = max_d c_max,d
    for (int d = 1; d < ndim; ++d) ch = fmax(ch, cm[d]);
    for (int d = 0; d < ndim; ++d) cm[d] = ch;
  }
  double dt;
  if (ctl->dt_fixed > 0.0) {
    dt = ctl->dt_fixed;
  } else {
    double worst = 0.0;
    for (int q = 0; q < ctl->ndx; ++q) {
      double s = 0.0;
      for (int d = 0; d < ndim; ++d) s = s + cm[d] / dxtab[3 * q + d];
      worst = fmax(worst, s);
    }
    dt = ctl->cfl / worst;
  }
  ctl->dt = dt;
  ctl->psi_decay = glm ? exp((-dt / GLM_CR) * ch) : 1.0;
  ctl->t += dt;
  for (int s = clear_lo; s <= clear_hi; ++s)
    for (int d = 0; d < 3; ++d) ctl->cm[s][d] = 0ull;
}

// Host-provided step controls, set on the stream (no host buffer lifetime).
__global__ void k_set_control(Control* ctl, double dt_fixed, double cfl, double t) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->dt_fixed = dt_fixed;
    ctl->cfl = cfl;
    ctl->t = t;
  }
}

// Copies the interior of every block from buffer `src` to buffer `dst`.
__global__ void __launch_bounds__(256) k_copy_interior(StateTable st, const Tile* tiles, int ntiles, int tx,
                                                     int ty, int tz, int nv, int src, int dst) {
  const int tcells = tx * ty * tz;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile tl = tiles[t];
    const BlockDev& B = st.blocks[tl.block];
    for (int c = threadIdx.x; c < tcells; c += 256) {
      const int i = tl.o[0] + c % tx, j = tl.o[1] + (c / tx) % ty, k = tl.o[2] + c / (tx * ty);
      if (i >= B.n[0] || j >= B.n[1] || k >= B.n[2]) continue;
      long long vs, ws;
      gptr p = cell_addr(st, B, src, i, j, k, vs);
      gptr_w q = cell_addr_w(st, B, dst, i, j, k, ws);
      for (int v = 0; v < nv; ++v) q[v * ws] = p[v * vs];
    }
  }
}

// Cell-centred current J = curl B of buffer `in` at every interior cell of
// the tile list, by fourth-order central differences (Sect. 4.4, eq. jcd4
// at cell centres) along each active direction; halos from the face
// neighbours (every face must have one).  Plane v of J at J + v * jplane.
template <int NDIM>
__global__ void __launch_bounds__(256) k_current(StateTable st, const Tile* tiles, int ntiles, int tx, int ty, int tz,
                                               int in, double* J, long long jplane) {
  const int tcells = tx * ty * tz;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile tl = tiles[t];
    const BlockDev& B = st.blocks[tl.block];
    for (int c = threadIdx.x; c < tcells; c += 256) {
      const int i = tl.o[0] + c % tx, j = tl.o[1] + (c / tx) % ty, k = tl.o[2] + c / (tx * ty);
      if (i >= B.n[0] || j >= B.n[1] || k >= B.n[2]) continue;
      double dB[3][3];   // dB[a][q] = d B_q / d x_a
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int q = 0; q < 3; ++q) dB[a][q] = 0.0;
      static_for<0, NDIM>([&](auto Ac) {
        constexpr int A = decltype(Ac)::value;
        double b[5][3];
#pragma unroll
        for (int s = -2; s <= 2; ++s) {
          if (s == 0) continue;
          int cc[3] = {i, j, k};
          cc[A] += s;
          load_cell_vars<5, 3, A>(st, tl.block, in, cc[0], cc[1], cc[2], b[s + 2]);
        }
#pragma unroll
        for (int q = 0; q < 3; ++q)
          dB[A][q] = (-1.0 * b[4][q] + 8.0 * b[3][q] - 8.0 * b[1][q] + b[0][q]) / (12.0 * B.dx[A]);
      });
      const long long o = B.coff + ((long long)k * B.n[1] + j) * B.n[0] + i;
      J[o] = dB[1][2] - dB[2][1];
      J[jplane + o] = dB[2][0] - dB[0][2];
      J[2 * jplane + o] = dB[0][1] - dB[1][0];
    }
  }
}

// Divergence of B by fourth-order central differences along each active
// direction (the monitor of Sect. 4.5.1), at every interior cell of the tile
// list, from buffer `in` with face neighbours' interiors (or fixed ghost
// layers) as halo.  Writes out[block] (interior layout) when out is set, and
// per tile the sum of |div B| over its cells, reduced in a fixed order.
template <int NDIM>
__global__ void __launch_bounds__(256) k_divb(StateTable st, const Tile* tiles, int ntiles, int tx, int ty, int tz,
                                            int in, double* const* out, double* tsum) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int tcells = tx * ty * tz;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile tl = tiles[t];
    const BlockDev& B = st.blocks[tl.block];
    double acc = 0.0;
    for (int c = tid; c < tcells; c += 256) {
      const int i = tl.o[0] + c % tx, j = tl.o[1] + (c / tx) % ty, k = tl.o[2] + c / (tx * ty);
      if (i >= B.n[0] || j >= B.n[1] || k >= B.n[2]) continue;
      double div = 0.0;
      static_for<0, NDIM>([&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        double b[5];
#pragma unroll
        for (int s = -2; s <= 2; ++s) {
          if (s == 0) continue;
          int cc[3] = {i, j, k};
          cc[D] += s;
          load_cell_vars<5 + D, 1, D>(st, tl.block, in, cc[0], cc[1], cc[2], &b[s + 2]);
        }
        div = div + (8.0 * (b[3] - b[1]) - (b[4] - b[0])) / (12.0 * B.dx[D]);
      });
      if (out) out[tl.block][((long long)k * B.n[1] + j) * B.n[0] + i] = div;
      acc = acc + fabs(div);
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) tsum[t] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
}

// Sum of n values in a fixed order (one work-group of 256 threads).
__global__ void __launch_bounds__(256) k_sum_fixed(const double* x, int n, double* result) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int q = tid; q < n; q += 256) acc = acc + x[q];
  acc = wave_sum(acc);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) *result = (red[0] + red[1]) + (red[2] + red[3]);
}

// Clears one c_max slot (used before a standalone c_max reduction).
__global__ void k_clear_slot(Control* ctl, int slot) {
  if (threadIdx.x < 3 && blockIdx.x == 0) ctl->cm[slot][threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------------------
// Variant table.
// ---------------------------------------------------------------------------

template <int NDIM, bool MHD, int TX, int TY, int TZ, int NT, int NGRP, int WPE, bool EMIT = false,
          bool RUNS = false, bool LIM = false, bool GLM = false, bool HALL = false, bool CORE = false>
static void launch_stage(const StageParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_stage<NDIM, MHD, TX, TY, TZ, NT, NGRP, WPE, EMIT, RUNS, LIM, GLM, HALL, CORE>),
                     dim3(grid), dim3(NT), 0, s, p);
}

// rec: the reconstruction (0 MP5, 1 LIM03)
#define AMRVAC_VARIANT(ND, M, TX, TY, TZ, NT, NGRP, WPE)                                          \
  {ND, M, 0, 0, TX, TY, TZ, NT, NGRP, WPE, (const void*)&k_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE>, \
   &launch_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE>,                                             \
   #ND "d-" #M "-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE}
// the same with interfaces evaluated in runs along each pencil
#define AMRVAC_VARIANT_R(ND, M, TX, TY, TZ, NT, NGRP, WPE)                                                     \
  {ND, M, 0, 0, TX, TY, TZ, NT, NGRP, WPE, (const void*)&k_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, false, true>, \
   &launch_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, false, true>,                                             \
   #ND "d-" #M "-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs"}
// the same with the owned cells' state kept in registers for the whole tile
#define AMRVAC_VARIANT_RC(ND, M, TX, TY, TZ, NT, NGRP, WPE)                                                  \
  {ND, M, 0, 0, TX, TY, TZ, NT, NGRP, WPE,                                                                   \
   (const void*)&k_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, false, true, false, false, false, true>,          \
   &launch_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, false, true, false, false, false, true>,                  \
   #ND "d-" #M "-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs-core"}
// GLM-MHD (physics code 2), MP5 or LIM03 (REC), in runs along each pencil
#define AMRVAC_VARIANT_G(ND, REC, TX, TY, TZ, NT, NGRP, WPE)                                                    \
  {ND, 2, REC, 0, TX, TY, TZ, NT, NGRP, WPE,                                                                       \
   (const void*)&k_stage<ND, true, TX, TY, TZ, NT, NGRP, WPE, false, true, (REC == 1), true>,                  \
   &launch_stage<ND, true, TX, TY, TZ, NT, NGRP, WPE, false, true, (REC == 1), true>,                          \
   #ND "d-glm-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs-rec" #REC}
// Hall MHD (physics MHD, eta_h > 0), MP5 or LIM03 (REC), in runs along each pencil
#define AMRVAC_VARIANT_H(ND, REC, TX, TY, TZ, NT, NGRP, WPE)                                                   \
  {ND, 1, REC, 1, TX, TY, TZ, NT, NGRP, WPE,                                                                   \
   (const void*)&k_stage<ND, true, TX, TY, TZ, NT, NGRP, WPE, false, true, (REC == 1), false, true>,          \
   &launch_stage<ND, true, TX, TY, TZ, NT, NGRP, WPE, false, true, (REC == 1), false, true>,                  \
   #ND "d-hall-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs-rec" #REC}
// LIM03 reconstruction in runs along each pencil
#define AMRVAC_VARIANT_LR(ND, M, TX, TY, TZ, NT, NGRP, WPE)                                                         \
  {ND, M, 1, 0, TX, TY, TZ, NT, NGRP, WPE, (const void*)&k_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, false, true, true>, \
   &launch_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, false, true, true>,                                             \
   #ND "d-" #M "-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs-lim03"}
// LIM03 reconstruction
#define AMRVAC_VARIANT_L(ND, M, TX, TY, TZ, NT, NGRP, WPE)                                                            \
  {ND, M, 1, 0, TX, TY, TZ, NT, NGRP, WPE, (const void*)&k_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, false, false, true>, \
   &launch_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, false, false, true>,                                             \
   #ND "d-" #M "-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-lim03"}

// Owned cells kept in registers for the whole tile (CORE), for LIM03, GLM
// and Hall MHD
#define AMRVAC_VARIANT_LRC(ND, M, TX, TY, TZ, NT, NGRP, WPE)                                                  \
  {ND, M, 1, 0, TX, TY, TZ, NT, NGRP, WPE,                                                                   \
   (const void*)&k_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, false, true, true, false, false, true>,           \
   &launch_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, false, true, true, false, false, true>,                   \
   #ND "d-" #M "-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs-lim03-core"}
#define AMRVAC_VARIANT_GC(ND, REC, TX, TY, TZ, NT, NGRP, WPE)                                                 \
  {ND, 2, REC, 0, TX, TY, TZ, NT, NGRP, WPE,                                                                 \
   (const void*)&k_stage<ND, true, TX, TY, TZ, NT, NGRP, WPE, false, true, (REC == 1), true, false, true>,   \
   &launch_stage<ND, true, TX, TY, TZ, NT, NGRP, WPE, false, true, (REC == 1), true, false, true>,           \
   #ND "d-glm-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs-rec" #REC "-core"}
#define AMRVAC_VARIANT_HC(ND, REC, TX, TY, TZ, NT, NGRP, WPE)                                                 \
  {ND, 1, REC, 1, TX, TY, TZ, NT, NGRP, WPE,                                                                 \
   (const void*)&k_stage<ND, true, TX, TY, TZ, NT, NGRP, WPE, false, true, (REC == 1), false, true, true>,   \
   &launch_stage<ND, true, TX, TY, TZ, NT, NGRP, WPE, false, true, (REC == 1), false, true, true>,           \
   #ND "d-hall-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs-rec" #REC "-core"}

// Tile shapes the autotuner chooses from (the first of each (ndim,
// physics) is the default).  WPE = minimum waves per SIMD requested from
// the register allocator.
static const StageVariant g_variants[] = {
    // 1D
    AMRVAC_VARIANT(1, false, 128, 1, 1, 128, 1, 1),
    AMRVAC_VARIANT(1, false, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT_RC(1, false, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT(1, true, 128, 1, 1, 128, 1, 1),
    AMRVAC_VARIANT(1, true, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT_R(1, true, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT_RC(1, true, 64, 1, 1, 64, 1, 1),
    // 2D
    AMRVAC_VARIANT(2, false, 16, 16, 1, 256, 1, 1),
    AMRVAC_VARIANT(2, false, 16, 16, 1, 256, 1, 3),
    AMRVAC_VARIANT(2, false, 32, 8, 1, 256, 1, 1),
    AMRVAC_VARIANT_R(2, false, 16, 16, 1, 256, 1, 1),
    AMRVAC_VARIANT_RC(2, false, 16, 16, 1, 256, 1, 2),
    AMRVAC_VARIANT(2, true, 16, 16, 1, 256, 2, 1),
    AMRVAC_VARIANT(2, true, 16, 16, 1, 256, 1, 1),
    AMRVAC_VARIANT(2, true, 16, 16, 1, 256, 2, 3),
    AMRVAC_VARIANT(2, true, 32, 8, 1, 256, 2, 1),
    AMRVAC_VARIANT_R(2, true, 16, 16, 1, 256, 1, 1),
    AMRVAC_VARIANT_R(2, true, 16, 16, 1, 256, 2, 2),
    AMRVAC_VARIANT_RC(2, true, 16, 16, 1, 256, 1, 2),
    AMRVAC_VARIANT_RC(2, true, 16, 16, 1, 256, 2, 2),
    // 3D: the owned-cell (CORE) forms first
    AMRVAC_VARIANT_RC(3, false, 8, 8, 4, 256, 1, 2),
    AMRVAC_VARIANT(3, false, 8, 8, 8, 512, 2, 1),
    AMRVAC_VARIANT(3, false, 8, 8, 4, 256, 1, 1),
    AMRVAC_VARIANT_R(3, false, 8, 8, 4, 256, 1, 2),
    AMRVAC_VARIANT_RC(3, true, 8, 8, 8, 512, 1, 2),
    AMRVAC_VARIANT_RC(3, true, 8, 8, 4, 256, 1, 2),
    AMRVAC_VARIANT_RC(3, true, 8, 4, 4, 128, 1, 2),
    AMRVAC_VARIANT_RC(3, true, 8, 8, 4, 256, 2, 3),
    AMRVAC_VARIANT_R(3, true, 8, 8, 4, 256, 2, 4),
    AMRVAC_VARIANT_R(3, true, 8, 8, 4, 256, 2, 3),
    AMRVAC_VARIANT_R(3, true, 8, 8, 8, 512, 2, 4),
    AMRVAC_VARIANT_R(3, true, 8, 8, 4, 256, 1, 2),
    AMRVAC_VARIANT(3, true, 8, 8, 4, 256, 2, 3),
    // LIM03 (the default of each (ndim, physics) first)
    AMRVAC_VARIANT_LR(1, true, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT_LRC(1, true, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT_LR(2, false, 16, 16, 1, 256, 1, 1),
    AMRVAC_VARIANT_LRC(2, false, 16, 16, 1, 256, 1, 2),
    AMRVAC_VARIANT_LR(2, true, 16, 16, 1, 256, 1, 1),
    AMRVAC_VARIANT_LR(2, true, 16, 16, 1, 256, 2, 2),
    AMRVAC_VARIANT_LRC(2, true, 16, 16, 1, 256, 1, 2),
    AMRVAC_VARIANT_LRC(3, false, 8, 8, 4, 256, 1, 2),
    AMRVAC_VARIANT_LR(3, false, 8, 8, 4, 256, 1, 2),
    AMRVAC_VARIANT_LRC(3, true, 8, 8, 4, 256, 1, 2),
    AMRVAC_VARIANT_LRC(3, true, 8, 8, 8, 512, 1, 2),
    AMRVAC_VARIANT_LR(3, true, 8, 8, 4, 256, 2, 4),
    AMRVAC_VARIANT_LR(3, true, 8, 8, 4, 256, 2, 3),
    AMRVAC_VARIANT_LR(3, true, 8, 8, 8, 512, 2, 4),
    AMRVAC_VARIANT_L(1, false, 128, 1, 1, 128, 1, 1),
    AMRVAC_VARIANT_L(1, false, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT_L(1, true, 128, 1, 1, 128, 1, 1),
    AMRVAC_VARIANT_L(1, true, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT_L(2, false, 16, 16, 1, 256, 1, 1),
    AMRVAC_VARIANT_L(2, false, 32, 8, 1, 256, 1, 1),
    AMRVAC_VARIANT_L(2, true, 16, 16, 1, 256, 2, 1),
    AMRVAC_VARIANT_L(2, true, 16, 16, 1, 256, 1, 1),
    AMRVAC_VARIANT_L(2, true, 32, 8, 1, 256, 2, 1),
    AMRVAC_VARIANT_L(3, false, 8, 8, 4, 256, 1, 1),
    AMRVAC_VARIANT_L(3, false, 8, 8, 8, 512, 2, 1),
    AMRVAC_VARIANT_L(3, true, 8, 8, 4, 256, 2, 3),
    // GLM-MHD
    AMRVAC_VARIANT_G(1, 0, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT_G(2, 0, 16, 16, 1, 256, 2, 2),
    AMRVAC_VARIANT_G(2, 0, 16, 16, 1, 256, 1, 1),
    AMRVAC_VARIANT_GC(2, 0, 16, 16, 1, 256, 1, 2),
    AMRVAC_VARIANT_GC(3, 0, 8, 8, 4, 256, 1, 2),
    AMRVAC_VARIANT_GC(3, 0, 8, 8, 8, 512, 1, 2),
    AMRVAC_VARIANT_GC(3, 0, 8, 8, 4, 256, 3, 3),
    AMRVAC_VARIANT_G(3, 0, 8, 8, 4, 256, 2, 3),
    AMRVAC_VARIANT_G(3, 0, 8, 8, 4, 256, 3, 4),
    AMRVAC_VARIANT_G(1, 1, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT_G(2, 1, 16, 16, 1, 256, 2, 2),
    AMRVAC_VARIANT_GC(3, 1, 8, 8, 4, 256, 1, 2),
    AMRVAC_VARIANT_G(3, 1, 8, 8, 4, 256, 2, 4),
    AMRVAC_VARIANT_G(3, 1, 8, 8, 4, 256, 2, 3),
    // Hall MHD
    AMRVAC_VARIANT_H(1, 0, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT_H(2, 0, 16, 16, 1, 256, 2, 2),
    AMRVAC_VARIANT_HC(3, 0, 8, 8, 4, 256, 1, 2),
    AMRVAC_VARIANT_H(3, 0, 8, 8, 4, 256, 2, 4),
    AMRVAC_VARIANT_H(3, 0, 8, 8, 4, 256, 2, 2),
    AMRVAC_VARIANT_H(1, 1, 64, 1, 1, 64, 1, 1),
    AMRVAC_VARIANT_H(2, 1, 16, 16, 1, 256, 2, 2),
    AMRVAC_VARIANT_HC(3, 1, 8, 8, 4, 256, 1, 2),
    AMRVAC_VARIANT_H(3, 1, 8, 8, 4, 256, 2, 4),
};

const StageVariant* stage_variants(int* count) {
  *count = (int)(sizeof(g_variants) / sizeof(g_variants[0]));
  return g_variants;
}

// Code-emitting stage kernels (the adjoint's forward recompute), one per
// (ndim, physics); their tile shapes match the adjoint kernels'.
#define AMRVAC_EMIT(ND, M, TX, TY, TZ, NT, NGRP, WPE)                                                          \
  {ND, M, 0, 0, TX, TY, TZ, NT, NGRP, WPE, (const void*)&k_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, true, true>, \
   &launch_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, true, true>,                                             \
   #ND "d-" #M "-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs-emit"}
#define AMRVAC_EMIT_L(ND, M, TX, TY, TZ, NT, NGRP, WPE)                                                             \
  {ND, M, 1, 0, TX, TY, TZ, NT, NGRP, WPE, (const void*)&k_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, true, true, true>, \
   &launch_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, true, true, true>,                                             \
   #ND "d-" #M "-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs-lim03-emit"}

#define AMRVAC_EMIT_C(ND, M, TX, TY, TZ, NT, NGRP, WPE)                                                       \
  {ND, M, 0, 0, TX, TY, TZ, NT, NGRP, WPE,                                                                   \
   (const void*)&k_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, true, true, false, false, false, true>,           \
   &launch_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, true, true, false, false, false, true>,                   \
   #ND "d-" #M "-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs-emit-core"}
#define AMRVAC_EMIT_LC(ND, M, TX, TY, TZ, NT, NGRP, WPE)                                                      \
  {ND, M, 1, 0, TX, TY, TZ, NT, NGRP, WPE,                                                                   \
   (const void*)&k_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, true, true, true, false, false, true>,            \
   &launch_stage<ND, M, TX, TY, TZ, NT, NGRP, WPE, true, true, true, false, false, true>,                    \
   #ND "d-" #M "-tile" #TX "x" #TY "x" #TZ "-nt" #NT "-g" #NGRP "-w" #WPE "-runs-lim03-emit-core"}

static const StageVariant g_emit[] = {
    AMRVAC_EMIT(1, false, 64, 1, 1, 64, 1, 1),
    AMRVAC_EMIT(1, true, 64, 1, 1, 64, 1, 1),
    AMRVAC_EMIT_C(2, false, 16, 16, 1, 256, 1, 2),
    AMRVAC_EMIT_C(2, true, 16, 16, 1, 256, 1, 2),
    AMRVAC_EMIT_C(3, false, 8, 8, 4, 256, 1, 2),
    AMRVAC_EMIT_C(3, true, 8, 8, 4, 256, 1, 2),
    AMRVAC_EMIT_L(1, false, 64, 1, 1, 64, 1, 1),
    AMRVAC_EMIT_L(1, true, 64, 1, 1, 64, 1, 1),
    AMRVAC_EMIT_LC(2, false, 16, 16, 1, 256, 1, 2),
    AMRVAC_EMIT_LC(2, true, 16, 16, 1, 256, 1, 2),
    AMRVAC_EMIT_LC(3, false, 8, 8, 4, 256, 1, 2),
    AMRVAC_EMIT_LC(3, true, 8, 8, 4, 256, 1, 2),
};

const StageVariant* emit_variant(int ndim, int mhd, int rec) {
  for (const StageVariant& v : g_emit)
    if (v.ndim == ndim && v.mhd == mhd && v.rec == rec) return &v;
  return nullptr;
}

template <int NDIM, bool MHD>
static void launch_cmax_t(const CmaxParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_cmax<NDIM, MHD>), dim3(grid), dim3(256), 0, s, p);
}

void launch_cmax(int ndim, int mhd, const CmaxParams& p, int grid, hipStream_t s) {
  if (ndim == 1) mhd ? launch_cmax_t<1, true>(p, grid, s) : launch_cmax_t<1, false>(p, grid, s);
  if (ndim == 2) mhd ? launch_cmax_t<2, true>(p, grid, s) : launch_cmax_t<2, false>(p, grid, s);
  if (ndim == 3) mhd ? launch_cmax_t<3, true>(p, grid, s) : launch_cmax_t<3, false>(p, grid, s);
}

void launch_step_begin(Control* ctl, const double* dxtab, int ndim, int glm, int clear_lo, int clear_hi,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(64), 0, s, ctl, dxtab, ndim, glm, clear_lo, clear_hi);
}

void launch_set_control(Control* ctl, double dt_fixed, double cfl, double t, hipStream_t s) {
  hipLaunchKernelGGL(k_set_control, dim3(1), dim3(64), 0, s, ctl, dt_fixed, cfl, t);
}

void launch_copy_interior(const StateTable& st, const Tile* tiles, int ntiles, int tx, int ty, int tz, int nv,
                          int src, int dst, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_interior, dim3(grid), dim3(256), 0, s, st, tiles, ntiles, tx, ty, tz, nv, src,
                     dst);
}

void launch_current(int ndim, const StateTable& st, const Tile* tiles, int ntiles, int tx, int ty, int tz, int in,
                    double* J, long long jplane, int grid, hipStream_t s) {
  if (ntiles <= 0) return;
  if (ndim == 1) hipLaunchKernelGGL(k_current<1>, dim3(grid), dim3(256), 0, s, st, tiles, ntiles, tx, ty, tz, in, J, jplane);
  if (ndim == 2) hipLaunchKernelGGL(k_current<2>, dim3(grid), dim3(256), 0, s, st, tiles, ntiles, tx, ty, tz, in, J, jplane);
  if (ndim == 3) hipLaunchKernelGGL(k_current<3>, dim3(grid), dim3(256), 0, s, st, tiles, ntiles, tx, ty, tz, in, J, jplane);
}

void launch_divb(int ndim, const StateTable& st, const Tile* tiles, int ntiles, int tx, int ty, int tz, int in,
                 double* const* out, double* tsum, double* total, int grid, hipStream_t s) {
  if (ndim == 1) hipLaunchKernelGGL(k_divb<1>, dim3(grid), dim3(256), 0, s, st, tiles, ntiles, tx, ty, tz, in, out, tsum);
  if (ndim == 2) hipLaunchKernelGGL(k_divb<2>, dim3(grid), dim3(256), 0, s, st, tiles, ntiles, tx, ty, tz, in, out, tsum);
  if (ndim == 3) hipLaunchKernelGGL(k_divb<3>, dim3(grid), dim3(256), 0, s, st, tiles, ntiles, tx, ty, tz, in, out, tsum);
  hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, tsum, ntiles, total);
}

void launch_clear_slot(Control* ctl, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_slot, dim3(1), dim3(64), 0, s, ctl, slot);
}

}  // namespace amrvac
