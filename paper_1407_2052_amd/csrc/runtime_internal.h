// Host runtime internals shared by runtime.cpp (forward path, C ABI) and
// adjoint.cpp (reverse mode).
#pragma once
#include "amrvac.h"
#include "amrvac_internal.h"

#include <map>
#include <string>
#include <vector>

namespace amrvac {

const StageVariant* stage_variants(int* count);
// Code-emitting stage kernel for (ndim, physics), or nullptr.
const StageVariant* emit_variant(int ndim, int mhd, int rec);
void launch_cmax(int ndim, int mhd, const CmaxParams& p, int grid, hipStream_t s);
void launch_current(int ndim, const StateTable& st, const Tile* tiles, int ntiles, int tx, int ty, int tz, int in,
                    double* J, long long jplane, int grid, hipStream_t s);
void launch_divb(int ndim, const StateTable& st, const Tile* tiles, int ntiles, int tx, int ty, int tz, int in,
                 double* const* out, double* tsum, double* total, int grid, hipStream_t s);
void launch_step_begin(Control* ctl, const double* dxtab, int ndim, int glm, int clear_lo, int clear_hi,
                       hipStream_t s);
void launch_clear_slot(Control* ctl, int slot, hipStream_t s);
void launch_set_control(Control* ctl, double dt_fixed, double cfl, double t, hipStream_t s);
void launch_copy_interior(const StateTable& st, const Tile* tiles, int ntiles, int tx, int ty, int tz, int nv,
                          int src, int dst, int grid, hipStream_t s);

// A range of the tile list that one batched stage launch covers.
struct LaunchGroup {
  int tile_begin, ntiles, grid;
};

struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace amrvac

// The context behind the opaque handle of the C ABI.
struct amrvac_ctx {
  using BlockDev = amrvac::BlockDev;
  using StageVariant = amrvac::StageVariant;
  using Tile = amrvac::Tile;
  using Control = amrvac::Control;
  using GraphEntry = amrvac::GraphEntry;

  amrvac_config cfg{};
  int nvar = 0;
  int exec = AMRVAC_EXEC_BATCHED;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  // the adjoint's second stream (recompute beside the reverse sweep) and its
  // events, created on first use
  hipStream_t adj_side = nullptr;
  hipEvent_t adj_ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int device = 0;
  int ncu = 0;
  std::string err;

  // blocks
  std::vector<amrvac_block> hb;
  std::vector<BlockDev> hdev;
  BlockDev* d_blocks = nullptr;
  long long total_cells = 0;    // interior cells of all blocks
  long long face_words[3] = {0, 0, 0};   // upper fixed-face cells per direction
  long long ghost_cells = 0;             // face ghost cells of all fixed faces
  long long slot_stride = 0;    // doubles per scratch slot

  // tiles of the chosen variant
  const StageVariant* var = nullptr;
  int var_index = 0;
  std::vector<Tile> htiles;
  Tile* d_tiles = nullptr;
  std::vector<int> blk_tile_begin, blk_tile_count;

  // dynamic grid activation: 1 = advanced, 0 = passive (kept, read as halo)
  std::vector<unsigned char> active;
  int n_active = 0;
  std::vector<Tile> hptiles;   // tiles of the passive blocks
  Tile* d_ptiles = nullptr;
  int grid_batched = 0;
  std::vector<amrvac::LaunchGroup> launch_groups;   // batched stage: one launch per group of size classes
  bool single_launch = false;                       // BATCHED_SINGLE: one group holding every class

  // scratch
  double* d_scr = nullptr;
  int nslots = 0;
  // amrvac_ssprk_step_noalloc: this device's fixed stage-buffer array
  // (resolved at amrvac_create; null if that failed), and the base the
  // state tables use while such a call enqueues (null: d_scr)
  double* noalloc_scr = nullptr;
  double* scr_override = nullptr;

  // control
  Control* d_ctl = nullptr;
  double* d_dxtab = nullptr;
  int ndx = 0;
  double** d_rhs_ptrs = nullptr;
  std::vector<double*> hrhs;
  // amrvac_divb: per-block output pointers, per-tile sums, total
  double** d_divb_ptrs = nullptr;
  std::vector<double*> hdivb;
  double* d_divb_sum = nullptr;   // divb_cap doubles (tiles + 1)
  double* d_J = nullptr;          // Hall MHD: current, 3 planes of total_cells
  int divb_cap = 0;

  std::map<int, GraphEntry> graphs;
};


namespace amrvac {
// Helpers implemented in runtime.cpp.
amrvac_status ctx_fail(amrvac_ctx* c, amrvac_status st, const char* fmt, ...);
amrvac_status ensure_slots(amrvac_ctx* c, int n);
StateTable state_table(const amrvac_ctx* c);
int scheme_stages(int scheme);
// One step of `scheme` with state buffer U (read), per-stage output buffers
// outs[1..s] (outs[s] receives U^{n+1}) and low-storage accumulator S.
// Stages launched by a code-emitting kernel on its own tile list, with the
// MP5 piece codes of L(stage input) of stage i written to codes[i - 1].
struct EmitPlan {
  const StageVariant* var;
  const Tile* tiles;
  int ntiles;
  int grid;
  unsigned char* codes[6];
  long long code_plane;
  double* cm_hist[6];   // c_max of stage i's input state is written to cm_hist[i - 1]
};
void enqueue_step_outs(amrvac_ctx* c, int scheme, int exec, hipStream_t s, int U, const int* outs, int S,
                       const EmitPlan* emit = nullptr);
void launch_cmax_of(amrvac_ctx* c, int buf, int slot, hipStream_t s);
amrvac_status read_status(amrvac_ctx* c);
// Shu-Osher table (Sect. 2.3) as used by the stage recipes: alpha[i][k],
// beta[i][k] for stages i = 1..s.
void scheme_table(int scheme, double alpha[6][6], double beta[6][6]);
}  // namespace amrvac
