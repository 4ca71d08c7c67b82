// Internal data structures shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace amrvac {

constexpr int NG = 3;          // ghost layers (MP5 stencils reach i-2..i+3)
constexpr int MAX_SLOTS = 8;   // c_max slots per step (stages + 1)

// One block as the kernels see it.
struct BlockDev {
  double* u;            // caller's padded state (buffer id 0)
  long long off;        // offset (doubles) of this block inside one scratch slot
  long long coff;       // offset (cells) of this block in per-cell arrays (off / nvar)
  long long cells;      // interior cells n0*n1*n2
  int n[3];             // interior extents (1 for inactive directions)
  int P[3];             // padded extents
  int g[3];             // ghost depth per direction (3 or 0)
  int nbr[6];           // face neighbours, -1 = fixed ghosts in u
  double dx[3];
  double inv_dx[3];
  // Adjoint bookkeeping of fixed faces (-1 where the face has a neighbour):
  // fco[d]: index, in 8-byte code words after the interior cells of a code
  //   plane, of the words of the interfaces on the upper face of direction d
  //   (one per face cell, transverse coordinates in x, y, z order);
  // gho[f]: index, in ghost cells of the boundary-data adjoint, of the 3
  //   ghost layers of face f (-x, +x, -y, +y, -z, +z), layer-major from the
  //   face outwards, transverse coordinates in x, y, z order.
  long long fco[3];
  long long gho[6];
};

// One unit of work: a box of interior cells of one block.
struct Tile {
  int block;
  int o[3];             // origin (interior coordinates)
};

// Device-resident step control: c_max slots (uint64 bit patterns of
// non-negative doubles, so integer max == floating max), dt, t, error flag.
struct Control {
  unsigned long long cm[MAX_SLOTS][3];
  double dt;
  double t;
  double dt_fixed;      // > 0: fixed step
  double cfl;
  int err;              // sticky: 1 = non-physical state met
  int ndx;              // number of distinct dx tuples in dxtab
  int pad[2];
  // c_max maximiser per direction ((block << 32) | interior linear index),
  // filled by the adjoint's argmax reduction
  long long arg[3];
  // GLM: factor exp(-dt c_h / c_r) of this step's psi decay
  double psi_decay;
};

// GLM: c_r = c_p^2 / c_h of the operator-split psi decay.
constexpr double GLM_CR = 0.18;

// Buffers: id 0 = caller's padded u; id k >= 1 = scratch slot k-1 with the
// interior-only layout, at scr + (k-1)*slot_stride + block.off.
struct StateTable {
  const BlockDev* blocks;
  double* scr;
  long long slot_stride;
};

constexpr int MAX_SRC = 3;

// Parameters of one fused stage launch:
//   L     = L(buffer `in`)   (c_max from slot cm_in)
//   dst   = sum_j a[j] * buffer src[j] + (dt * b) * L          (mode 0)
//   sdst  = sum_j sa[j] * buffer ssrc[j] + (dt * sb) * L       (optional)
//   rhs_out[block] = L  (interior layout)                     (mode 1)
// Every WG keeps a running maximum of |v_d| + c_f,d of the new state and
// folds it into slot cm_out at exit (cm_out < 0: none).  cm_reset >= 0:
// one thread clears that slot.
struct StageParams {
  StateTable st;
  const Tile* tiles;
  int tile_begin;
  int ntiles;
  Control* ctl;
  double gamma;
  int in;
  int mode;
  int cm_in, cm_out, cm_reset;
  int nsrc;
  int src[MAX_SRC];
  double a[MAX_SRC];
  double b;
  int dst;
  int snsrc;
  int ssrc[MAX_SRC];
  double sa[MAX_SRC];
  double sb;
  int sdst;
  double* const* rhs_out;
  // GLM: multiply psi by the step's decay factor (last stage of a step)
  int decay_psi;
  // Hall MHD: eta_h and the cell-centred current of the input state, three
  // planes of interior cells (plane v at J + v * jplane, block at coff)
  double eta_h;
  const double* J;
  long long jplane;
  // Optional (only the code-emitting kernels write it): linear-piece codes
  // of the reconstructions (MP5 or LIM03) of L(in), one byte per
  // (direction, cell, variable) for the
  // interface on the cell's lower face, low nibble for the F+ stencil and
  // high nibble for the F- stencil, at
  //   codes + D * code_plane + (block.coff + cell) * 8 + v.
  unsigned char* codes;
  long long code_plane;
  // words of the upper fixed-face interfaces start at word code_faces of a
  // plane (the number of interior cells)
  long long code_faces;
  // Optional (the adjoint's recompute): the c_max of this stage's input
  // state (slot cm_in as read at launch) is copied to cm_hist[0..2]
  double* cm_hist;
};

// One compiled form of the fused stage kernel (a tile shape and its
// options): its table entry, shared by the kernel file that instantiates it
// and the runtime that selects it.
struct StageVariant {
  int ndim, mhd, rec, hall, tx, ty, tz, nt, ngrp, wpe;   // mhd: physics code; rec: 0 MP5, 1 LIM03
  const void* fn;
  void (*launch)(const StageParams&, int grid, hipStream_t);
  const char* name;
};

struct CmaxParams {
  StateTable st;
  const Tile* tiles;
  int ntiles;
  int tx, ty, tz;       // tile extents used for the tile list
  Control* ctl;
  double gamma;
  int in;
  int slot;
  double eta_h;         // Hall MHD: the whistler speed enters c_max
};

// One fixed face of a block list (the adjoint's boundary-data pass).
struct FixedFace {
  int block;
  int face;   // 2 d + side
};

constexpr int MAX_TERMS = 6;

// Parameters of one vector-Jacobian product of L (adjoint of one stage
// state U = buffer `in`):
//   mu   = sum_q mu_a[q]  * buffer mu_src[q]                (on the fly)
//   dst  = sum_q lam_a[q] * buffer lam_src[q] + scale * J_L(U)^T mu
// for the local dependence of L on U; the MP5 linear pieces come from the
// codes the forward recompute of U's stage wrote (layout as in
// StageParams).  The c_max part (through the maximising cell) is added by a
// separate reduction from the per-tile sums written to cpart[tile*3+d].
struct VjpParams {
  StateTable st;
  const Tile* tiles;
  int ntiles;
  Control* ctl;
  double gamma;
  int in;
  const unsigned char* codes;
  long long code_plane;
  long long code_faces;   // as in StageParams
  int recon;   // reconstruction the codes refer to: 0 MP5, 1 LIM03
  int nmu;
  int mu_src[MAX_TERMS];
  double mu_a[MAX_TERMS];
  int nlam;
  int lam_src[MAX_TERMS];
  double lam_a[MAX_TERMS];
  int dst;
  double scale;
  // c_max of the state `in` per direction, as its recompute recorded it; the
  // VJP marks the maximising cells (lowest (block, cell) key, atomicMin into
  // ctl->arg, which the c_max term then consumes and resets)
  const double* cm_in;
  double* cpart;    // per-work-group c_max adjoint partials, 3 per work-group
};

// A VJP kernel (tile shape as the code-emitting stage kernel of the same
// ndim and physics), its c_max-term kernel and its fixed-face ghost kernel.
struct VjpVariant {
  int ndim, mhd, tx, ty, tz, nt;
  const void* fn;
  void (*launch)(const VjpParams&, int grid, hipStream_t);
  // the c_max term: sum of the partials, applied at the maximising cell
  void (*cmax_term)(StateTable, int, const double*, int, Control*, double, int, int, double, hipStream_t);
  void (*ghost)(const VjpParams&, const FixedFace*, int, double*, long long, double*, int, hipStream_t);
};

// dst = sum_j a[j] * src[j] over the interiors (up to 6 terms).
struct CombineParams {
  StateTable st;
  const Tile* tiles;
  int ntiles, tx, ty, tz, nv;
  int n;
  int src[6];
  double a[6];
  int dst;
};

const VjpVariant* vjp_variant(int ndim, int mhd);
void launch_combine(const CombineParams& p, int grid, hipStream_t s);
void launch_lam_import(StateTable st, double* const* ptrs, int nv, int dst, int nblocks, hipStream_t s);
void launch_lam_export(StateTable st, double* const* ptrs, int nv, int src, int nblocks, const double* gadj,
                       long long gplane, hipStream_t s);

}  // namespace amrvac
