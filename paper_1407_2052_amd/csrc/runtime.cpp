// Host runtime behind the C ABI of include/amrvac.h: argument validation,
// block and tile tables, context-owned scratch, Shu-Osher stage recipes
// (Sect. 2.3), per-block and batched (persistent, graph-replayed, one launch
// per block-size class or one per stage) execution.
#include "amrvac.h"
#include "amrvac_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "runtime_internal.h"

using namespace amrvac;

static const char* g_noctx_error = "";

// Stage buffers of amrvac_ssprk_step_noalloc: one fixed array per device,
// held until the process ends.  Host code never passes `scratch` itself to a
// kernel (in host code the name is a stand-in, not a device address): the
// address on each device is resolved once with hipGetSymbolAddress, with
// that device current, and kept in g_scratch_addr.
static __device__ __align__(256) double scratch[AMRVAC_NOALLOC_MAX_DOUBLES];
static std::mutex g_scratch_mu;
static std::map<int, double*> g_scratch_addr;

static hipError_t scratch_address(int device, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
  g_scratch_addr[device] = static_cast<double*>(p);
  *out = static_cast<double*>(p);
  return hipSuccess;
}

static amrvac_status fail(amrvac_ctx* c, amrvac_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

#define HIP_TRY(ctx, expr)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(ctx, e_ == hipErrorOutOfMemory ? AMRVAC_ERR_NOMEM : AMRVAC_ERR_DEVICE,       \
                  "%s failed: %s", #expr, hipGetErrorString(e_));                              \
  } while (0)

static void drop_graphs(amrvac_ctx* c) {
  for (auto& kv : c->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  c->graphs.clear();
}

static void free_tables(amrvac_ctx* c) {
  if (c->d_blocks) (void)hipFree(c->d_blocks);
  if (c->d_tiles) (void)hipFree(c->d_tiles);
  if (c->d_scr) (void)hipFree(c->d_scr);
  if (c->d_dxtab) (void)hipFree(c->d_dxtab);
  if (c->d_rhs_ptrs) (void)hipFree(c->d_rhs_ptrs);
  if (c->d_ptiles) (void)hipFree(c->d_ptiles);
  if (c->d_divb_ptrs) (void)hipFree(c->d_divb_ptrs);
  if (c->d_J) (void)hipFree(c->d_J);
  c->d_J = nullptr;
  if (c->d_divb_sum) (void)hipFree(c->d_divb_sum);
  c->d_divb_ptrs = nullptr;
  c->d_divb_sum = nullptr;
  c->divb_cap = 0;
  c->d_ptiles = nullptr;
  c->d_blocks = nullptr;
  c->d_tiles = nullptr;
  c->d_scr = nullptr;
  c->d_dxtab = nullptr;
  c->d_rhs_ptrs = nullptr;
  c->nslots = 0;
}

// ---------------------------------------------------------------------------
// Tables
// ---------------------------------------------------------------------------
static uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  auto spread = [](uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
  };
  return spread(x) | (spread(y) << 1) | (spread(z) << 2);
}

static int count_variants(const amrvac_ctx* c) {
  int nv = 0, k = 0;
  const StageVariant* v = stage_variants(&nv);
  for (int i = 0; i < nv; ++i)
    if (v[i].ndim == c->cfg.ndim && v[i].mhd == c->cfg.physics && v[i].rec == c->cfg.recon &&
        v[i].hall == (c->cfg.eta_h > 0.0))
      ++k;
  return k;
}

static const StageVariant* pick_variant(const amrvac_ctx* c, int want) {
  int nv = 0;
  const StageVariant* v = stage_variants(&nv);
  int k = 0;
  for (int i = 0; i < nv; ++i) {
    if (v[i].ndim == c->cfg.ndim && v[i].mhd == c->cfg.physics && v[i].rec == c->cfg.recon &&
        v[i].hall == (c->cfg.eta_h > 0.0)) {
      if (k == want) return &v[i];
      ++k;
    }
  }
  return nullptr;
}

static amrvac_status select_variant(amrvac_ctx* c, int i);

// Build the tile list of the current variant: blocks ordered largest first,
// then along a Morton curve of their origins; tiles of a block contiguous and
// Morton-ordered.  The list is cut into launch groups of whole size classes
// (blocks of equal cell count), one stage launch per group; the single-launch
// form keeps every class in one group.
static amrvac_status build_tiles(amrvac_ctx* c) {
  const StageVariant* V = c->var;
  const int T[3] = {V->tx, V->ty, V->tz};
  const int nb = (int)c->hb.size();
  int per_cu = 0;
  HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, V->fn, V->nt, 0));
  if (per_cu < 1) return fail(c, AMRVAC_ERR_DEVICE, "stage kernel cannot be resident");
  const long long resident = (long long)per_cu * c->ncu;
  auto active_tiles = [&](int b) -> long long {
    if (!(c->active.empty() || c->active[b])) return 0;
    long long k = 1;
    for (int d = 0; d < 3; ++d) k *= (c->hb[b].n[d] + T[d] - 1) / T[d];
    return k;
  };
  std::vector<int> order(nb);
  std::vector<uint64_t> key(nb);
  std::vector<long long> cells(nb);
  for (int b = 0; b < nb; ++b) {
    order[b] = b;
    const amrvac_block& q = c->hb[b];
    uint32_t o[3] = {0, 0, 0};
    for (int d = 0; d < c->cfg.ndim; ++d) {
      double x = q.xlo[d] / q.dx[d];
      long long xi = (long long)std::llround(x) + (1ll << 20);
      o[d] = (uint32_t)std::max(0ll, std::min(xi, (1ll << 21) - 1));
    }
    key[b] = morton3(o[0], o[1], o[2]);
    cells[b] = (long long)q.n[0] * q.n[1] * q.n[2];
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (cells[a] != cells[b]) return cells[a] > cells[b];
    return key[a] < key[b];
  });
  // Launch groups.  The persistent schedule gives XCD x the x-th eighth of a
  // launch's tiles, and a tile of a small block costs more than one of a
  // large block (larger halo per cell, more fixed faces), so a launch over
  // mixed classes loads the XCDs unevenly; one launch per class keeps every
  // launch uniform and the tiles an XCD shares its L2 over compact in space.
  // A class too small to fill the chip twice over joins the next one (a
  // trailing one the previous group); inside a group of several classes each
  // class is dealt out in 8 Morton-contiguous parts, part x of every class in
  // the x-th eighth, so every XCD holds an eighth of each class.
  std::vector<std::pair<size_t, size_t>> groups;   // [begin, end) in `order`
  {
    std::vector<std::pair<size_t, size_t>> classes;
    std::vector<long long> ctiles;
    for (size_t a = 0; a < order.size();) {
      size_t e = a;
      long long k = 0;
      while (e < order.size() && cells[order[e]] == cells[order[a]]) k += active_tiles(order[e++]);
      classes.push_back({a, e});
      ctiles.push_back(k);
      a = e;
    }
    std::vector<std::vector<size_t>> gcls;   // classes of each group
    long long acc = 0;
    for (size_t k = 0; k < classes.size(); ++k) {
      if (gcls.empty() || (acc >= 2 * resident && !c->single_launch)) {
        gcls.push_back({});
        acc = 0;
      }
      gcls.back().push_back(k);
      acc += ctiles[k];
    }
    if (gcls.size() > 1 && acc < 2 * resident) {
      for (size_t k : gcls.back()) gcls[gcls.size() - 2].push_back(k);
      gcls.pop_back();
    }
    std::vector<int> dealt;
    dealt.reserve(nb);
    for (auto& g : gcls) {
      const size_t begin = dealt.size();
      for (int part = 0; part < 8; ++part)
        for (size_t k : g) {
          const size_t n = classes[k].second - classes[k].first;
          for (size_t q = classes[k].first + n * part / 8; q < classes[k].first + n * (part + 1) / 8; ++q)
            dealt.push_back(order[q]);
        }
      groups.push_back({begin, dealt.size()});
    }
    order.swap(dealt);
  }
  c->htiles.clear();
  c->hptiles.clear();
  c->blk_tile_begin.assign(nb, 0);
  c->blk_tile_count.assign(nb, 0);
  c->launch_groups.clear();
  size_t gi = 0;
  for (size_t oi = 0; oi < order.size(); ++oi) {
    const int b = order[oi];
    if (oi == groups[gi].first) c->launch_groups.push_back({(int)c->htiles.size(), 0, 0});
    if (oi + 1 == groups[gi].second) ++gi;
    const amrvac_block& q = c->hb[b];
    const bool act = c->active.empty() || c->active[b];
    int nt[3];
    for (int d = 0; d < 3; ++d) nt[d] = (q.n[d] + T[d] - 1) / T[d];
    std::vector<std::pair<uint64_t, Tile>> tl;
    for (int z = 0; z < nt[2]; ++z)
      for (int y = 0; y < nt[1]; ++y)
        for (int x = 0; x < nt[0]; ++x) {
          Tile t;
          t.block = b;
          t.o[0] = x * T[0];
          t.o[1] = y * T[1];
          t.o[2] = z * T[2];
          tl.push_back({morton3(x, y, z), t});
        }
    std::stable_sort(tl.begin(), tl.end(),
                     [](const std::pair<uint64_t, Tile>& a, const std::pair<uint64_t, Tile>& b) {
                       return a.first < b.first;
                     });
    if (!act) {   // passive: no work, its tiles only feed the slot copies
      c->blk_tile_begin[b] = (int)c->htiles.size();
      for (auto& p : tl) c->hptiles.push_back(p.second);
      continue;
    }
    c->blk_tile_begin[b] = (int)c->htiles.size();
    c->blk_tile_count[b] = (int)tl.size();
    for (auto& p : tl) c->htiles.push_back(p.second);
  }
  if (c->htiles.empty()) return fail(c, AMRVAC_ERR_INVALID, "no active block");
  if (c->d_tiles) (void)hipFree(c->d_tiles);
  c->d_tiles = nullptr;
  HIP_TRY(c, hipMalloc(&c->d_tiles, sizeof(Tile) * c->htiles.size()));
  HIP_TRY(c, hipMemcpyAsync(c->d_tiles, c->htiles.data(), sizeof(Tile) * c->htiles.size(),
                            hipMemcpyHostToDevice, c->stream));
  if (c->d_ptiles) (void)hipFree(c->d_ptiles);
  c->d_ptiles = nullptr;
  if (!c->hptiles.empty()) {
    HIP_TRY(c, hipMalloc(&c->d_ptiles, sizeof(Tile) * c->hptiles.size()));
    HIP_TRY(c, hipMemcpyAsync(c->d_ptiles, c->hptiles.data(), sizeof(Tile) * c->hptiles.size(),
                              hipMemcpyHostToDevice, c->stream));
  }
  c->grid_batched = (int)std::min<long long>(resident, (long long)c->htiles.size());
  {
    std::vector<LaunchGroup> kept;
    for (size_t g = 0; g < c->launch_groups.size(); ++g) {
      LaunchGroup L = c->launch_groups[g];
      const int end = g + 1 < c->launch_groups.size() ? c->launch_groups[g + 1].tile_begin : (int)c->htiles.size();
      L.ntiles = end - L.tile_begin;
      L.grid = (int)std::min<long long>(resident, (long long)L.ntiles);
      if (L.ntiles > 0) kept.push_back(L);
    }
    c->launch_groups.swap(kept);
  }
  // the tile list is copied from host memory that lives in the context
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return AMRVAC_OK;
}

namespace amrvac {
amrvac_status ensure_slots(amrvac_ctx* c, int n) {
  if (c->nslots >= n) return AMRVAC_OK;
  drop_graphs(c);
  if (c->d_scr) (void)hipFree(c->d_scr);
  c->d_scr = nullptr;
  c->nslots = 0;
  size_t bytes = sizeof(double) * (size_t)c->slot_stride * (size_t)n;
  HIP_TRY(c, hipMalloc(&c->d_scr, bytes));
  c->nslots = n;
  return AMRVAC_OK;
}
}  // namespace amrvac

static amrvac_status select_variant(amrvac_ctx* c, int i) {
  const StageVariant* v = pick_variant(c, i);
  if (!v) return fail(c, AMRVAC_ERR_INVALID, "variant %d does not exist", i);
  if (v == c->var && !c->htiles.empty()) return AMRVAC_OK;
  drop_graphs(c);
  c->var = v;
  c->var_index = i;
  if (c->hb.empty()) return AMRVAC_OK;
  return build_tiles(c);
}

namespace amrvac {
StateTable state_table(const amrvac_ctx* c) {
  StateTable st;
  st.blocks = c->d_blocks;
  st.scr = c->scr_override ? c->scr_override : c->d_scr;
  st.slot_stride = c->slot_stride;
  return st;
}
}  // namespace amrvac

// ---------------------------------------------------------------------------
// Stage recipes (Sect. 2.3).  Buffer ids: 0 = caller's u (U^n on entry,
// U^{n+1} on exit); 1 = A, 2 = B, 3 = S (scratch slots 0..2).
// ---------------------------------------------------------------------------
struct Recipe {
  int in;
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
};

namespace amrvac {
int scheme_stages(int scheme) { return scheme == AMRVAC_RK3 ? 3 : scheme == AMRVAC_SSPRK43 ? 4 : 5; }
}  // namespace amrvac

// SSPRK(5,4) coefficients as printed (Sect. 2.3.2); alpha_50 renormalised so
// the row sums to one.
static const double A20 = 0.44437049406734, A21 = 0.55562950593266;
static const double A30 = 0.62010185138540, A32 = 0.37989814861460;
static const double A40 = 0.17807995410773, A43 = 0.82192004589227;
static const double A52 = 0.51723167208978, A53 = 0.12759831133288, A54 = 0.34833675773694;
static const double B10 = 0.39175222700392, B21 = 0.36841059262959, B32 = 0.25189177424738;
static const double B43 = 0.54497475021237, B53 = 0.08460416338212, B54 = 0.22600748319395;

static Recipe rc(int in, std::initializer_list<std::pair<int, double>> srcs, double b, int dst) {
  Recipe r{};
  r.in = in;
  r.nsrc = 0;
  for (auto& s : srcs) {
    r.src[r.nsrc] = s.first;
    r.a[r.nsrc] = s.second;
    ++r.nsrc;
  }
  r.b = b;
  r.dst = dst;
  r.sdst = -1;
  r.snsrc = 0;
  return r;
}

static Recipe with_s(Recipe r, std::initializer_list<std::pair<int, double>> srcs, double sb, int sdst) {
  r.snsrc = 0;
  for (auto& s : srcs) {
    r.ssrc[r.snsrc] = s.first;
    r.sa[r.snsrc] = s.second;
    ++r.snsrc;
  }
  r.sb = sb;
  r.sdst = sdst;
  return r;
}

// Stage recipes with state buffer U (the step's input, read only), per-stage
// output buffers outs[1..s] (outs[s] receives U^{n+1}) and the low-storage
// accumulator S (SSPRK(5,4) only).
static std::vector<Recipe> recipes(int scheme, int U, const int* o, int S) {
  std::vector<Recipe> r;
  if (scheme == AMRVAC_RK3) {
    r.push_back(rc(U, {{U, 1.0}}, 1.0, o[1]));
    r.push_back(rc(o[1], {{U, 0.75}, {o[1], 0.25}}, 0.25, o[2]));
    r.push_back(rc(o[2], {{U, 1.0 / 3.0}, {o[2], 2.0 / 3.0}}, 2.0 / 3.0, o[3]));
  } else if (scheme == AMRVAC_SSPRK43) {
    r.push_back(rc(U, {{U, 1.0}}, 0.5, o[1]));
    r.push_back(rc(o[1], {{o[1], 1.0}}, 0.5, o[2]));
    r.push_back(rc(o[2], {{U, 2.0 / 3.0}, {o[2], 1.0 / 3.0}}, 1.0 / 6.0, o[3]));
    r.push_back(rc(o[3], {{o[3], 1.0}}, 0.5, o[4]));
  } else {
    const double A50 = 1.0 - (A52 + A53 + A54);
    r.push_back(rc(U, {{U, 1.0}}, B10, o[1]));                                 // U1
    r.push_back(rc(o[1], {{U, A20}, {o[1], A21}}, B21, o[2]));                 // U2
    r.push_back(with_s(rc(o[2], {{U, A30}, {o[2], A32}}, B32, o[3]),           // U3
                       {{U, A50}, {o[2], A52}}, 0.0, S));                      // S = a50 U0 + a52 U2
    r.push_back(with_s(rc(o[3], {{U, A40}, {o[3], A43}}, B43, o[4]),           // U4
                       {{S, 1.0}, {o[3], A53}}, B53, S));                      // S += a53 U3 + dt b53 L(U3)
    r.push_back(rc(o[4], {{S, 1.0}, {o[4], A54}}, B54, o[5]));                 // U5
  }
  return r;
}

namespace amrvac {
void scheme_table(int scheme, double alpha[6][6], double beta[6][6]) {
  for (int i = 0; i < 6; ++i)
    for (int k = 0; k < 6; ++k) alpha[i][k] = beta[i][k] = 0.0;
  if (scheme == AMRVAC_RK3) {
    alpha[1][0] = 1.0; beta[1][0] = 1.0;
    alpha[2][0] = 0.75; alpha[2][1] = 0.25; beta[2][1] = 0.25;
    alpha[3][0] = 1.0 / 3.0; alpha[3][2] = 2.0 / 3.0; beta[3][2] = 2.0 / 3.0;
  } else if (scheme == AMRVAC_SSPRK43) {
    alpha[1][0] = 1.0; beta[1][0] = 0.5;
    alpha[2][1] = 1.0; beta[2][1] = 0.5;
    alpha[3][0] = 2.0 / 3.0; alpha[3][2] = 1.0 / 3.0; beta[3][2] = 1.0 / 6.0;
    alpha[4][3] = 1.0; beta[4][3] = 0.5;
  } else {
    alpha[1][0] = 1.0; beta[1][0] = B10;
    alpha[2][0] = A20; alpha[2][1] = A21; beta[2][1] = B21;
    alpha[3][0] = A30; alpha[3][2] = A32; beta[3][2] = B32;
    alpha[4][0] = A40; alpha[4][3] = A43; beta[4][3] = B43;
    alpha[5][0] = 1.0 - (A52 + A53 + A54); alpha[5][2] = A52; alpha[5][3] = A53; alpha[5][4] = A54;
    beta[5][3] = B53; beta[5][4] = B54;
  }
}
}  // namespace amrvac

static StageParams make_params(const amrvac_ctx* c, const Recipe& r, int cm_in, int cm_out,
                               int cm_reset) {
  StageParams p{};
  p.st = state_table(c);
  p.tiles = c->d_tiles;
  p.tile_begin = 0;
  p.ntiles = (int)c->htiles.size();
  p.ctl = c->d_ctl;
  p.gamma = c->cfg.gamma;
  p.in = r.in;
  p.mode = 0;
  p.cm_in = cm_in;
  p.cm_out = cm_out;
  p.cm_reset = cm_reset;
  p.nsrc = r.nsrc;
  for (int q = 0; q < MAX_SRC; ++q) {
    p.src[q] = q < r.nsrc ? r.src[q] : 0;
    p.a[q] = q < r.nsrc ? r.a[q] : 0.0;
    p.ssrc[q] = q < r.snsrc ? r.ssrc[q] : 0;
    p.sa[q] = q < r.snsrc ? r.sa[q] : 0.0;
  }
  p.b = r.b;
  p.dst = r.dst;
  p.snsrc = r.snsrc;
  p.sb = r.sb;
  p.sdst = r.sdst;
  p.rhs_out = nullptr;
  p.eta_h = c->cfg.eta_h;
  p.J = c->d_J;
  p.jplane = c->total_cells;
  return p;
}

// Hall MHD: the current of buffer `buf` on every interior cell (active and
// passive blocks), before a stage reads it.
static void launch_current_of(amrvac_ctx* c, int buf, hipStream_t s) {
  if (!(c->cfg.eta_h > 0.0)) return;
  const StateTable st = state_table(c);
  const int nt = (int)c->htiles.size(), np = (int)c->hptiles.size();
  launch_current(c->cfg.ndim, st, c->d_tiles, nt, c->var->tx, c->var->ty, c->var->tz, buf, c->d_J, c->total_cells,
                 std::max(1, std::min(nt, c->ncu * 8)), s);
  launch_current(c->cfg.ndim, st, c->d_ptiles, np, c->var->tx, c->var->ty, c->var->tz, buf, c->d_J, c->total_cells,
                 std::max(1, std::min(np, c->ncu * 8)), s);
}

// Launch one stage in the context's execution form.
static void launch_stage(amrvac_ctx* c, StageParams p, int exec, hipStream_t s) {
  launch_current_of(c, p.in, s);
  if (exec == AMRVAC_EXEC_BATCHED) {
    for (size_t g = 0; g < c->launch_groups.size(); ++g) {
      StageParams q = p;
      q.tile_begin = c->launch_groups[g].tile_begin;
      q.ntiles = c->launch_groups[g].ntiles;
      if (g > 0) q.cm_reset = -1;   // the slot reset runs in the first launch only
      c->var->launch(q, c->launch_groups[g].grid, s);
    }
    return;
  }
  const int nb = (int)c->hb.size();
  for (int b = 0; b < nb; ++b) {
    StageParams q = p;
    q.tile_begin = c->blk_tile_begin[b];
    q.ntiles = c->blk_tile_count[b];
    // the slot reset must run once, on the first launch only
    if (b > 0) q.cm_reset = -1;
    if (q.ntiles > 0) {
      c->var->launch(q, q.ntiles, s);
    } else if (b == 0 && p.cm_reset >= 0) {
      launch_clear_slot(c->d_ctl, p.cm_reset, s);   // block 0 is passive: clear here
    }
  }
}

namespace amrvac {
void launch_cmax_of(amrvac_ctx* c, int buf, int slot, hipStream_t s) {
  CmaxParams q{};
  q.st = state_table(c);
  q.tiles = c->d_tiles;
  q.ntiles = (int)c->htiles.size();
  q.tx = c->var->tx;
  q.ty = c->var->ty;
  q.tz = c->var->tz;
  q.ctl = c->d_ctl;
  q.gamma = c->cfg.gamma;
  q.in = buf;
  q.slot = slot;
  q.eta_h = c->cfg.eta_h;
  launch_clear_slot(c->d_ctl, slot, s);
  int grid = (int)std::min<long long>((long long)c->ncu * 8, (long long)c->htiles.size());
  // psi enters no wave speed: GLM uses the MHD reduction
  launch_cmax(c->cfg.ndim, c->cfg.physics != AMRVAC_HD, q, grid, s);
}
}  // namespace amrvac

// One step: dt, then the s stages.  c_max slots: slot 0 holds c_max(U^n);
// stage i (1-based) reads slot i-1 and accumulates slot i (slot 0 for the
// last stage, giving c_max(U^{n+1}) for the next step); stage 2 clears slot
// 0 once stage 1 no longer needs it.
namespace amrvac {
void enqueue_step_outs(amrvac_ctx* c, int scheme, int exec, hipStream_t s, int U, const int* outs, int S,
                       const EmitPlan* emit) {
  const int ns = scheme_stages(scheme);
  launch_step_begin(c->d_ctl, c->d_dxtab, c->cfg.ndim, c->cfg.physics == AMRVAC_GLM, 1, ns - 1, s);
  std::vector<Recipe> r = recipes(scheme, U, outs, S);
  for (int i = 1; i <= ns; ++i) {
    const int cm_in = i - 1;
    const int cm_out = (i == ns) ? 0 : i;
    const int cm_reset = (i == 2) ? 0 : -1;
    StageParams p = make_params(c, r[i - 1], cm_in, cm_out, cm_reset);
    p.decay_psi = (i == ns && c->cfg.physics == AMRVAC_GLM) ? 1 : 0;
    if (emit) {
      p.tiles = emit->tiles;
      p.tile_begin = 0;
      p.ntiles = emit->ntiles;
      p.codes = emit->codes[i - 1];
      p.code_plane = emit->code_plane;
      p.code_faces = c->total_cells;
      p.cm_hist = emit->cm_hist[i - 1];
      emit->var->launch(p, emit->grid, s);
    } else {
      launch_stage(c, p, exec, s);
    }
  }
}
}  // namespace amrvac

// Ping-pong form: stages alternate between A and B, the last writes out.
static void enqueue_step(amrvac_ctx* c, int scheme, int exec, hipStream_t s, int U, int A, int Bf, int S,
                         int out) {
  const int ns = scheme_stages(scheme);
  int outs[6];
  for (int i = 1; i <= ns; ++i) outs[i] = (i == ns) ? out : ((i % 2) ? A : Bf);
  enqueue_step_outs(c, scheme, exec, s, U, outs, S);
}

namespace amrvac {
amrvac_status read_status(amrvac_ctx* c) {
  int err = 0;
  HIP_TRY(c, hipMemcpyAsync(&err, &c->d_ctl->err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (err) {
    int zero = 0;
    HIP_TRY(c, hipMemcpy(&c->d_ctl->err, &zero, sizeof(int), hipMemcpyHostToDevice));
    return fail(c, AMRVAC_ERR_NONPHYSICAL, "non-physical state (rho <= 0, p <= 0 or non-finite)");
  }
  return AMRVAC_OK;
}

amrvac_status ctx_fail(amrvac_ctx* c, amrvac_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}
}  // namespace amrvac

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
static bool config_ok(const amrvac_config* cfg) {
  return cfg && cfg->ndim >= 1 && cfg->ndim <= 3 &&
         (cfg->physics == AMRVAC_HD || cfg->physics == AMRVAC_MHD || cfg->physics == AMRVAC_GLM) &&
         (cfg->exec == AMRVAC_EXEC_PER_BLOCK || cfg->exec == AMRVAC_EXEC_BATCHED ||
          cfg->exec == AMRVAC_EXEC_BATCHED_SINGLE) &&
         (cfg->recon == AMRVAC_MP5 || cfg->recon == AMRVAC_LIM03) &&
         std::isfinite(cfg->eta_h) && cfg->eta_h >= 0.0 && (cfg->eta_h == 0.0 || cfg->physics == AMRVAC_MHD) &&
         std::isfinite(cfg->gamma) && cfg->gamma > 1.0;
}

// Host-only validation shared by amrvac_set_blocks and
// amrvac_validate_blocks; writes the first violation into msg.
static bool blocks_ok(int nd, const amrvac_block* blocks, int nblocks, std::string& msg) {
  char buf[256];
  auto bad = [&](const char* fmt, int a, int b2, int c2) {
    snprintf(buf, sizeof(buf), fmt, a, b2, c2);
    msg = buf;
    return false;
  };
  if (!blocks || nblocks < 1) return bad("no blocks (%d %d %d)", nblocks, 0, 0);
  for (int b = 0; b < nblocks; ++b) {
    const amrvac_block& q = blocks[b];
    if (!q.u) return bad("block %d: u is NULL%s", b, 0, 0);
    for (int d = 0; d < 3; ++d) {
      if (d < nd) {
        if (q.n[d] < NG) return bad("block %d: n[%d] = %d < 3", b, d, q.n[d]);
        if (!std::isfinite(q.dx[d]) || !(q.dx[d] > 0.0))
          return bad("block %d: dx[%d] must be finite and > 0 (%d)", b, d, 0);
        for (int s = 0; s < 2; ++s) {
          int nb = q.nbr[2 * d + s];
          if (nb < -1 || nb >= nblocks) return bad("block %d: neighbour %d = %d out of range", b, 2 * d + s, nb);
          if (nb >= 0) {
            const amrvac_block& r = blocks[nb];
            if (r.nbr[2 * d + (1 - s)] != b)
              return bad("block %d face %d: neighbour %d does not point back", b, 2 * d + s, nb);
            for (int e = 0; e < nd; ++e)
              if (e != d && r.n[e] != q.n[e])
                return bad("block %d face %d: face size differs from block %d", b, 2 * d + s, nb);
          }
        }
      } else {
        if (q.n[d] != 1) return bad("block %d: n[%d] must be 1 for an inactive direction (%d)", b, d, q.n[d]);
        if (q.nbr[2 * d] != -1 || q.nbr[2 * d + 1] != -1)
          return bad("block %d: inactive direction %d has neighbours (%d)", b, d, 0);
      }
    }
  }
  return true;
}

extern "C" {

int amrvac_abi_version(void) { return AMRVAC_ABI_VERSION; }

amrvac_status amrvac_create(const amrvac_config* cfg, void* hip_stream, amrvac_ctx** out) {
  if (!out) {
    g_noctx_error = "amrvac_create: out is NULL";
    return AMRVAC_ERR_INVALID;
  }
  *out = nullptr;
  if (!cfg) {
    g_noctx_error = "amrvac_create: cfg is NULL";
    return AMRVAC_ERR_INVALID;
  }
  if (!config_ok(cfg)) {
    g_noctx_error = "amrvac_create: invalid config (ndim 1..3, physics HD/MHD/GLM, exec, recon, gamma > 1, eta_h >= 0 with MHD only)";
    return AMRVAC_ERR_INVALID;
  }
  amrvac_ctx* c = new amrvac_ctx();
  c->cfg = *cfg;
  c->exec = cfg->exec == AMRVAC_EXEC_BATCHED_SINGLE ? AMRVAC_EXEC_BATCHED : cfg->exec;
  c->single_launch = cfg->exec == AMRVAC_EXEC_BATCHED_SINGLE;
  c->nvar = cfg->physics == AMRVAC_GLM ? 9 : cfg->physics == AMRVAC_MHD ? 8 : 2 + cfg->ndim;
  c->stream = (hipStream_t)hip_stream;
  c->var = pick_variant(c, 0);
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&c->d_ctl, sizeof(Control));
  if (e == hipSuccess) e = hipMemset(c->d_ctl, 0, sizeof(Control));
  if (e == hipSuccess && scratch_address(c->device, &c->noalloc_scr) != hipSuccess) {
    c->noalloc_scr = nullptr;   // amrvac_ssprk_step_noalloc reports DEVICE
    (void)hipGetLastError();
  }
  if (e != hipSuccess || !c->var) {
    g_noctx_error = "amrvac_create: HIP device setup failed";
    if (c->d_ctl) (void)hipFree(c->d_ctl);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
    return e == hipErrorOutOfMemory ? AMRVAC_ERR_NOMEM : AMRVAC_ERR_DEVICE;
  }
  *out = c;
  return AMRVAC_OK;
}

amrvac_status amrvac_validate_blocks(const amrvac_config* cfg, const amrvac_block* blocks, int nblocks,
                                     char* msg, int msglen) {
  std::string m;
  amrvac_status st = AMRVAC_OK;
  if (!config_ok(cfg)) {
    m = "invalid config (ndim 1..3, physics HD/MHD/GLM, exec, recon, gamma > 1, eta_h >= 0 with MHD only)";
    st = AMRVAC_ERR_INVALID;
  } else if (!blocks_ok(cfg->ndim, blocks, nblocks, m)) {
    st = AMRVAC_ERR_INVALID;
  }
  if (msg && msglen > 0) {
    snprintf(msg, (size_t)msglen, "%s", m.c_str());
  }
  return st;
}

amrvac_status amrvac_set_blocks(amrvac_ctx* c, const amrvac_block* blocks, int nblocks) {
  if (!c) return AMRVAC_ERR_INVALID;
  const int nd = c->cfg.ndim;
  {
    std::string m;
    if (!blocks_ok(nd, blocks, nblocks, m)) return fail(c, AMRVAC_ERR_INVALID, "set_blocks: %s", m.c_str());
    if (c->cfg.eta_h > 0.0)
      for (int b = 0; b < nblocks; ++b)
        for (int d = 0; d < nd; ++d)
          if (blocks[b].nbr[2 * d] < 0 || blocks[b].nbr[2 * d + 1] < 0)
            return fail(c, AMRVAC_ERR_INVALID, "set_blocks: Hall MHD needs a neighbour on every face (block %d)", b);
  }
  drop_graphs(c);
  free_tables(c);
  c->hb.assign(blocks, blocks + nblocks);
  c->hdev.resize(nblocks);
  c->active.assign(nblocks, 1);
  c->n_active = nblocks;
  long long off = 0;
  std::vector<double> dxt;
  for (int b = 0; b < nblocks; ++b) {
    const amrvac_block& q = blocks[b];
    BlockDev& D = c->hdev[b];
    D.u = q.u;
    D.cells = (long long)q.n[0] * q.n[1] * q.n[2];
    D.off = off;
    D.coff = off / c->nvar;
    off += D.cells * c->nvar;
    for (int d = 0; d < 3; ++d) {
      D.n[d] = q.n[d];
      D.g[d] = d < nd ? NG : 0;
      D.P[d] = q.n[d] + 2 * D.g[d];
      D.dx[d] = d < nd ? q.dx[d] : 1.0;
      D.inv_dx[d] = 1.0 / D.dx[d];
    }
    for (int f = 0; f < 6; ++f) D.nbr[f] = q.nbr[f];
    bool seen = false;
    for (size_t k = 0; k < dxt.size(); k += 3)
      if (dxt[k] == D.dx[0] && dxt[k + 1] == D.dx[1] && dxt[k + 2] == D.dx[2]) seen = true;
    if (!seen) {
      dxt.push_back(D.dx[0]);
      dxt.push_back(D.dx[1]);
      dxt.push_back(D.dx[2]);
    }
  }
  c->total_cells = off / c->nvar;
  // fixed faces: code words of upper boundary interfaces, ghost cells of the
  // boundary-data adjoint
  for (int d = 0; d < 3; ++d) c->face_words[d] = 0;
  c->ghost_cells = 0;
  for (int b = 0; b < nblocks; ++b) {
    BlockDev& D = c->hdev[b];
    for (int d = 0; d < 3; ++d) {
      long long area = 1;
      for (int e = 0; e < 3; ++e)
        if (e != d) area *= D.n[e];
      D.fco[d] = (d < nd && D.nbr[2 * d + 1] < 0) ? c->face_words[d] : -1;
      if (D.fco[d] >= 0) c->face_words[d] += area;
      for (int side = 0; side < 2; ++side) {
        const int f = 2 * d + side;
        D.gho[f] = (d < nd && D.nbr[f] < 0) ? c->ghost_cells : -1;
        if (D.gho[f] >= 0) c->ghost_cells += 3 * area;
      }
    }
  }
  if (c->cfg.eta_h > 0.0)   // Hall MHD: the current of every interior cell, three planes
    HIP_TRY(c, hipMalloc(&c->d_J, sizeof(double) * 3 * (size_t)c->total_cells));
  c->slot_stride = (off + 31) / 32 * 32;
  c->ndx = (int)(dxt.size() / 3);
  HIP_TRY(c, hipMalloc(&c->d_blocks, sizeof(BlockDev) * nblocks));
  HIP_TRY(c, hipMemcpyAsync(c->d_blocks, c->hdev.data(), sizeof(BlockDev) * nblocks,
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMalloc(&c->d_dxtab, sizeof(double) * dxt.size()));
  HIP_TRY(c, hipMemcpyAsync(c->d_dxtab, dxt.data(), sizeof(double) * dxt.size(), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMalloc(&c->d_rhs_ptrs, sizeof(double*) * nblocks));
  amrvac_status st = build_tiles(c);
  if (st != AMRVAC_OK) return st;
  // control: ndx
  Control h{};
  HIP_TRY(c, hipMemcpyAsync(&h, c->d_ctl, sizeof(Control), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  h.ndx = c->ndx;
  HIP_TRY(c, hipMemcpy(c->d_ctl, &h, sizeof(Control), hipMemcpyHostToDevice));
  return AMRVAC_OK;
}

amrvac_status amrvac_set_exec(amrvac_ctx* c, int exec) {
  if (!c) return AMRVAC_ERR_INVALID;
  if (exec != AMRVAC_EXEC_PER_BLOCK && exec != AMRVAC_EXEC_BATCHED && exec != AMRVAC_EXEC_BATCHED_SINGLE)
    return fail(c, AMRVAC_ERR_INVALID, "set_exec: unknown execution form %d", exec);
  const bool single = exec == AMRVAC_EXEC_BATCHED_SINGLE;
  c->exec = single ? AMRVAC_EXEC_BATCHED : exec;
  if (exec != AMRVAC_EXEC_PER_BLOCK && single != c->single_launch) {
    // the launch grouping is part of the work list
    c->single_launch = single;
    drop_graphs(c);
    if (!c->hb.empty()) return build_tiles(c);
  }
  return AMRVAC_OK;
}

int amrvac_num_variants(const amrvac_ctx* c) { return c ? count_variants(c) : 0; }

const char* amrvac_variant_name(const amrvac_ctx* c, int i) {
  if (!c) return nullptr;
  const StageVariant* v = pick_variant(c, i);
  return v ? v->name : nullptr;
}

int amrvac_get_variant(const amrvac_ctx* c) { return c ? c->var_index : -1; }

amrvac_status amrvac_set_variant(amrvac_ctx* c, int i) {
  if (!c) return AMRVAC_ERR_INVALID;
  if (i < 0 || i >= count_variants(c)) return fail(c, AMRVAC_ERR_INVALID, "set_variant: %d out of range", i);
  return select_variant(c, i);
}

amrvac_status amrvac_autotune(amrvac_ctx* c, int scheme, int nsteps, double* ms_out) {
  if (!c) return AMRVAC_ERR_INVALID;
  if (c->hb.empty()) return fail(c, AMRVAC_ERR_INVALID, "autotune: no blocks set");
  if (scheme < AMRVAC_RK3 || scheme > AMRVAC_SSPRK54 || nsteps < 1)
    return fail(c, AMRVAC_ERR_INVALID, "autotune: invalid scheme or nsteps");
  if (c->n_active < (int)c->hb.size())
    return fail(c, AMRVAC_ERR_UNSUPPORTED, "autotune: some blocks are passive");
  const int nv = count_variants(c);
  if (ms_out)
    for (int i = 0; i < nv; ++i) ms_out[i] = -1.0;
  // cache lookup
  char key[256];
  hipDeviceProp_t prop;
  HIP_TRY(c, hipGetDeviceProperties(&prop, c->device));
  snprintf(key, sizeof(key), "%s|%d|%d|%d|%zu|%lld|%d|%d", prop.gcnArchName, c->cfg.ndim, c->cfg.physics,
           c->cfg.recon, c->hb.size(), c->total_cells, scheme, c->single_launch ? 1 : 0);
  const char* cache = std::getenv("AMRVAC_TUNE_CACHE");
  if (cache && *cache) {
    std::ifstream in(cache);
    std::string line;
    std::string found;
    while (std::getline(in, line)) {
      size_t sp = line.rfind(' ');
      if (sp != std::string::npos && line.substr(0, sp) == key) found = line.substr(sp + 1);
    }
    if (!found.empty())
      for (int i = 0; i < nv; ++i)
        if (found == pick_variant(c, i)->name) return select_variant(c, i);
  }
  // time every shape on scratch copies: slot ids 1..3 = A, B, S; 4 = U copy
  amrvac_status st = ensure_slots(c, 4);
  if (st != AMRVAC_OK) return st;
  const int keep = c->var_index;
  const int keep_exec = c->exec;
  c->exec = AMRVAC_EXEC_BATCHED;
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  int best = keep;
  float best_ms = 1e30f;
  for (int i = 0; i < nv; ++i) {
    st = select_variant(c, i);
    if (st != AMRVAC_OK) continue;
    launch_copy_interior(state_table(c), c->d_tiles, (int)c->htiles.size(), c->var->tx, c->var->ty, c->var->tz,
                         c->nvar, 0, 4, std::min<int>(c->ncu * 8, (int)c->htiles.size()), c->stream);
    launch_set_control(c->d_ctl, 0.0, 0.4, 0.0, c->stream);
    launch_cmax_of(c, 4, 0, c->stream);
    enqueue_step(c, scheme, AMRVAC_EXEC_BATCHED, c->stream, 4, 1, 2, 3, 4);   // warm-up
    HIP_TRY(c, hipEventRecord(e0, c->stream));
    for (int it = 0; it < nsteps; ++it) enqueue_step(c, scheme, AMRVAC_EXEC_BATCHED, c->stream, 4, 1, 2, 3, 4);
    HIP_TRY(c, hipEventRecord(e1, c->stream));
    HIP_TRY(c, hipEventSynchronize(e1));
    if (hipGetLastError() != hipSuccess) continue;
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
    ms /= nsteps;
    if (ms_out) ms_out[i] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = i;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->exec = keep_exec;
  st = read_status(c);
  if (st != AMRVAC_OK) {
    select_variant(c, keep);
    return st;
  }
  st = select_variant(c, best);
  if (st == AMRVAC_OK && cache && *cache) {
    std::ofstream out(cache, std::ios::app);
    out << key << " " << c->var->name << "\n";
  }
  return st;
}

amrvac_status amrvac_fd_rhs(amrvac_ctx* c, double* const* rhs, double* cmax_out) {
  if (!c) return AMRVAC_ERR_INVALID;
  if (c->hb.empty()) return fail(c, AMRVAC_ERR_INVALID, "fd_rhs: no blocks set");
  if (!rhs) return fail(c, AMRVAC_ERR_INVALID, "fd_rhs: rhs is NULL");
  const int nb = (int)c->hb.size();
  for (int b = 0; b < nb; ++b)
    if (!rhs[b]) return fail(c, AMRVAC_ERR_INVALID, "fd_rhs: rhs[%d] is NULL", b);
  c->hrhs.assign(rhs, rhs + nb);
  HIP_TRY(c, hipMemcpyAsync(c->d_rhs_ptrs, c->hrhs.data(), sizeof(double*) * nb, hipMemcpyHostToDevice,
                            c->stream));
  launch_cmax_of(c, 0, 0, c->stream);
  Recipe r = rc(0, {{0, 1.0}}, 0.0, 0);
  StageParams p = make_params(c, r, 0, -1, -1);
  p.mode = 1;
  p.rhs_out = c->d_rhs_ptrs;
  launch_stage(c, p, c->exec, c->stream);
  HIP_TRY(c, hipGetLastError());
  if (cmax_out) {
    unsigned long long cm[3];
    HIP_TRY(c, hipMemcpyAsync(cm, c->d_ctl->cm[0], sizeof(cm), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int d = 0; d < 3; ++d) {
      double v;
      std::memcpy(&v, &cm[d], sizeof(double));
      cmax_out[d] = v;
    }
    if (c->cfg.physics == AMRVAC_GLM) {   // c_h in every direction
      double ch = cmax_out[0];
      for (int d = 1; d < c->cfg.ndim; ++d) ch = std::max(ch, cmax_out[d]);
      for (int d = 0; d < c->cfg.ndim; ++d) cmax_out[d] = ch;
    }
    return read_status(c);
  }
  return AMRVAC_OK;
}

amrvac_status amrvac_divb(amrvac_ctx* c, double* const* out, double* mean_abs_out) {
  if (!c) return AMRVAC_ERR_INVALID;
  if (c->hb.empty()) return fail(c, AMRVAC_ERR_INVALID, "divb: no blocks set");
  if (c->cfg.physics == AMRVAC_HD) return fail(c, AMRVAC_ERR_INVALID, "divb: hydro has no magnetic field");
  const int nb = (int)c->hb.size();
  if (out)
    for (int b = 0; b < nb; ++b)
      if (!out[b]) return fail(c, AMRVAC_ERR_INVALID, "divb: out[%d] is NULL", b);
  const int nt = (int)c->htiles.size();
  if (!c->d_divb_ptrs) HIP_TRY(c, hipMalloc(&c->d_divb_ptrs, sizeof(double*) * nb));
  if (c->divb_cap < nt + 1) {   // the tile list changes with the variant and the active set
    if (c->d_divb_sum) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      (void)hipFree(c->d_divb_sum);
      c->d_divb_sum = nullptr;
      c->divb_cap = 0;
    }
    HIP_TRY(c, hipMalloc(&c->d_divb_sum, sizeof(double) * (nt + 1)));
    c->divb_cap = nt + 1;
  }
  if (out) {
    c->hdivb.assign(out, out + nb);
    HIP_TRY(c, hipMemcpyAsync(c->d_divb_ptrs, c->hdivb.data(), sizeof(double*) * nb, hipMemcpyHostToDevice,
                              c->stream));
  }
  const int grid = std::max(1, std::min(nt, c->ncu * 8));
  launch_divb(c->cfg.ndim, state_table(c), c->d_tiles, nt, c->var->tx, c->var->ty, c->var->tz, 0,
              out ? c->d_divb_ptrs : nullptr, c->d_divb_sum, c->d_divb_sum + nt, grid, c->stream);
  HIP_TRY(c, hipGetLastError());
  if (mean_abs_out) {
    double total = 0.0;
    HIP_TRY(c, hipMemcpyAsync(&total, c->d_divb_sum + nt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    long long cells = 0;
    for (int b = 0; b < nb; ++b)
      if (c->active[b]) cells += (long long)c->hb[b].n[0] * c->hb[b].n[1] * c->hb[b].n[2];
    *mean_abs_out = total / (double)cells;
  }
  return AMRVAC_OK;
}

static amrvac_status check_step_args(amrvac_ctx* c, int scheme, double cfl, const double* dt_fixed,
                                     int nsteps) {
  if (c->hb.empty()) return fail(c, AMRVAC_ERR_INVALID, "ssprk_step: no blocks set");
  if (scheme < AMRVAC_RK3 || scheme > AMRVAC_SSPRK54)
    return fail(c, AMRVAC_ERR_INVALID, "ssprk_step: unknown scheme %d", scheme);
  if (nsteps < 0) return fail(c, AMRVAC_ERR_INVALID, "ssprk_step: nsteps < 0");
  if (dt_fixed) {
    if (!std::isfinite(*dt_fixed) || !(*dt_fixed > 0.0))
      return fail(c, AMRVAC_ERR_INVALID, "ssprk_step: dt must be finite and > 0");
  } else if (!std::isfinite(cfl) || !(cfl > 0.0)) {
    return fail(c, AMRVAC_ERR_INVALID, "ssprk_step: cfl must be finite and > 0");
  }
  return AMRVAC_OK;
}

// Steps per graph of the multi-step graph: a graph launch costs about 6 us
// on top of its kernels (2D Euler 256^2: 81 us per step replaying a one-step
// graph, 75 us launching the kernels one by one, 74 us replaying 8-step
// graphs), so runs of steps replay 8-step graphs and the remainder the
// one-step graph.
constexpr int GRAPH_STEPS = 8;
constexpr int GRAPH_MULTI_KEY = 16;   // graphs[scheme + GRAPH_MULTI_KEY]: the multi-step graph

// The steps of amrvac_ssprk_step on the stage buffers the state tables
// point at (context scratch, or the fixed array); with use_graph the batched
// form replays cached graphs of GRAPH_STEPS steps and of one step.
static amrvac_status enqueue_steps(amrvac_ctx* c, int scheme, double cfl, const double* dt_fixed, int nsteps,
                                   double* t_inout, bool use_graph) {
  if (!c->hptiles.empty() && nsteps > 0) {
    // passive blocks: their current state in the stage buffers A and B,
    // which active neighbours read as halo at every stage
    const StageVariant* V = c->var;
    const int np = (int)c->hptiles.size();
    const int grid = std::max(1, std::min(np, c->ncu * 8));
    launch_copy_interior(state_table(c), c->d_ptiles, np, V->tx, V->ty, V->tz, c->nvar, 0, 1, grid, c->stream);
    launch_copy_interior(state_table(c), c->d_ptiles, np, V->tx, V->ty, V->tz, c->nvar, 0, 2, grid, c->stream);
  }
  launch_set_control(c->d_ctl, dt_fixed ? *dt_fixed : 0.0, cfl, t_inout ? *t_inout : 0.0, c->stream);
  if (nsteps > 0) launch_cmax_of(c, 0, 0, c->stream);
  const int exec = c->exec;
  if (use_graph && exec == AMRVAC_EXEC_BATCHED && nsteps > 0) {
    // both graphs are captured on first use, so a later longer call does
    // not capture inside its own run
    auto capture = [&](GraphEntry& g, int steps) -> amrvac_status {
      HIP_TRY(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
      for (int k = 0; k < steps; ++k) enqueue_step(c, scheme, exec, c->cap, 0, 1, 2, 3, 0);
      hipError_t e = hipStreamEndCapture(c->cap, &g.graph);
      if (e != hipSuccess) {
        g.graph = nullptr;
        return fail(c, AMRVAC_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
      }
      HIP_TRY(c, hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
      return AMRVAC_OK;
    };
    GraphEntry& g1 = c->graphs[scheme];
    GraphEntry& gm = c->graphs[scheme + GRAPH_MULTI_KEY];
    if (!g1.exec || !gm.exec) {
      amrvac_status st = g1.exec ? AMRVAC_OK : capture(g1, 1);
      if (st == AMRVAC_OK && !gm.exec) st = capture(gm, GRAPH_STEPS);
      if (st != AMRVAC_OK) return st;
    }
    int it = 0;
    for (; it + GRAPH_STEPS <= nsteps; it += GRAPH_STEPS) HIP_TRY(c, hipGraphLaunch(gm.exec, c->stream));
    for (; it < nsteps; ++it) HIP_TRY(c, hipGraphLaunch(g1.exec, c->stream));
  } else {
    for (int it = 0; it < nsteps; ++it) enqueue_step(c, scheme, exec, c->stream, 0, 1, 2, 3, 0);
  }
  HIP_TRY(c, hipGetLastError());
  return AMRVAC_OK;
}

// Reads the end time (synchronising) and the sticky device status.
static amrvac_status report_time(amrvac_ctx* c, double* t_inout) {
  if (!t_inout) return AMRVAC_OK;
  double t = 0.0;
  HIP_TRY(c, hipMemcpyAsync(&t, &c->d_ctl->t, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  amrvac_status st = read_status(c);
  *t_inout = t;
  return st;
}

amrvac_status amrvac_ssprk_step(amrvac_ctx* c, int scheme, double cfl, const double* dt_fixed,
                                int nsteps, double* t_inout) {
  if (!c) return AMRVAC_ERR_INVALID;
  amrvac_status st = check_step_args(c, scheme, cfl, dt_fixed, nsteps);
  if (st != AMRVAC_OK) return st;
  st = ensure_slots(c, 3);
  if (st != AMRVAC_OK) return st;
  st = enqueue_steps(c, scheme, cfl, dt_fixed, nsteps, t_inout, true);
  if (st != AMRVAC_OK) return st;
  return report_time(c, t_inout);
}

amrvac_status amrvac_ssprk_step_noalloc(amrvac_ctx* c, int scheme, double cfl, const double* dt_fixed,
                                        int nsteps, double* t_inout) {
  if (!c) return AMRVAC_ERR_INVALID;
  amrvac_status st = check_step_args(c, scheme, cfl, dt_fixed, nsteps);
  if (st != AMRVAC_OK) return st;
  if (!c->noalloc_scr)
    return fail(c, AMRVAC_ERR_DEVICE, "ssprk_step_noalloc: the fixed stage-buffer array has no address on device %d",
                c->device);
  const long long need = 3 * c->slot_stride;
  if (need > (long long)AMRVAC_NOALLOC_MAX_DOUBLES)
    return fail(c, AMRVAC_ERR_INVALID,
                "ssprk_step_noalloc: the stage buffers need %lld doubles, more than the %lld of the fixed array",
                need, (long long)AMRVAC_NOALLOC_MAX_DOUBLES);
  c->scr_override = c->noalloc_scr;
  st = enqueue_steps(c, scheme, cfl, dt_fixed, nsteps, t_inout, false);
  c->scr_override = nullptr;
  if (st != AMRVAC_OK) return st;
  return report_time(c, t_inout);
}

int amrvac_activation_flags(const amrvac_block* blocks, int nblocks, const unsigned char* want, int safety,
                            unsigned char* active_out) {
  if (!blocks || nblocks < 1 || !want || safety < 0 || !active_out) return -1;
  for (int b = 0; b < nblocks; ++b)
    for (int f = 0; f < 6; ++f)
      if (blocks[b].nbr[f] < -1 || blocks[b].nbr[f] >= nblocks) return -1;
  // step 1: the caller's criterion; step 2, `safety` times: a passive block
  // with an active face neighbour becomes active
  std::vector<unsigned char> cur(nblocks), next;
  for (int b = 0; b < nblocks; ++b) cur[b] = want[b] ? 1 : 0;
  for (int pass = 0; pass < safety; ++pass) {
    next = cur;
    for (int b = 0; b < nblocks; ++b) {
      if (cur[b]) continue;
      for (int f = 0; f < 6; ++f) {
        const int nb = blocks[b].nbr[f];
        if (nb >= 0 && cur[nb]) next[b] = 1;
      }
    }
    cur.swap(next);
  }
  int n = 0;
  for (int b = 0; b < nblocks; ++b) {
    active_out[b] = cur[b];
    n += cur[b];
  }
  return n;
}

amrvac_status amrvac_set_active(amrvac_ctx* c, const unsigned char* active) {
  if (!c) return AMRVAC_ERR_INVALID;
  if (c->hb.empty()) return fail(c, AMRVAC_ERR_INVALID, "set_active: no blocks set");
  const int nb = (int)c->hb.size();
  std::vector<unsigned char> a(nb, 1);
  int n = nb;
  if (active) {
    n = 0;
    for (int b = 0; b < nb; ++b) {
      a[b] = active[b] ? 1 : 0;
      n += a[b];
    }
  }
  if (n == 0) return fail(c, AMRVAC_ERR_INVALID, "set_active: no active block");
  drop_graphs(c);
  c->active = a;
  c->n_active = n;
  amrvac_status st = build_tiles(c);
  if (st != AMRVAC_OK) return st;
  // dt rule over the active blocks' cell widths
  std::vector<double> dxt;
  for (int b = 0; b < nb; ++b) {
    if (!a[b]) continue;
    const BlockDev& D = c->hdev[b];
    bool seen = false;
    for (size_t k = 0; k < dxt.size(); k += 3)
      if (dxt[k] == D.dx[0] && dxt[k + 1] == D.dx[1] && dxt[k + 2] == D.dx[2]) seen = true;
    if (!seen) {
      dxt.push_back(D.dx[0]);
      dxt.push_back(D.dx[1]);
      dxt.push_back(D.dx[2]);
    }
  }
  if (c->d_dxtab) (void)hipFree(c->d_dxtab);
  c->d_dxtab = nullptr;
  HIP_TRY(c, hipMalloc(&c->d_dxtab, sizeof(double) * dxt.size()));
  HIP_TRY(c, hipMemcpyAsync(c->d_dxtab, dxt.data(), sizeof(double) * dxt.size(), hipMemcpyHostToDevice,
                            c->stream));
  c->ndx = (int)(dxt.size() / 3);
  Control h{};
  HIP_TRY(c, hipMemcpyAsync(&h, c->d_ctl, sizeof(Control), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  h.ndx = c->ndx;
  HIP_TRY(c, hipMemcpy(c->d_ctl, &h, sizeof(Control), hipMemcpyHostToDevice));
  return AMRVAC_OK;
}

amrvac_status amrvac_sync(amrvac_ctx* c) {
  if (!c) return AMRVAC_ERR_INVALID;
  return read_status(c);
}

const char* amrvac_last_error(const amrvac_ctx* c) {
  if (!c) return g_noctx_error;
  return c->err.c_str();
}

void amrvac_destroy(amrvac_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  free_tables(c);
  if (c->d_ctl) (void)hipFree(c->d_ctl);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->adj_side) {
    (void)hipStreamSynchronize(c->adj_side);
    (void)hipStreamDestroy(c->adj_side);
  }
  for (hipEvent_t e : c->adj_ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
