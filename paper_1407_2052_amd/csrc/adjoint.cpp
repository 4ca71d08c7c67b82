// Reverse mode of the SSPRK time integration (Porth et al. 2014, Sect. 2.3)
// with checkpoint-and-recompute: amrvac_ssprk_adjoint.
//
// Forward map of one step (Shu-Osher form):
//   U(0) = U^n,  U(i) = sum_{k<i} alpha_ik U(k) + dt beta_ik L(U(k)),  U^{n+1} = U(s).
// Reverse of one step, given lam(s) = dJ/dU^{n+1}, for k = s-1 .. 0:
//   mu      = sum_{i>k} beta_ik lam(i)
//   lam(k)  = sum_{i>k} alpha_ik lam(i) + dt J_L(U(k))^T mu
// and dJ/dU^n = lam(0).  Every lam(i), i > k, is complete when stage k is
// processed, so each stage state costs exactly one vector-Jacobian product.
//
// Memory: checkpoints of U every ckpt_every steps; a segment is recomputed
// from its checkpoint with every stage state stored, together with the MP5
// linear-piece codes of L at each of them (8 bytes per cell and direction),
// then reversed.  On small lists (launches of at most two work-groups per
// CU) the next segment is recomputed on a second stream, into a second set
// of stage states and codes, while the current one is reversed.
#include "runtime_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>


using namespace amrvac;

namespace {

struct Adj {
  amrvac_ctx* c;
  const VjpVariant* V;
  std::vector<Tile> htiles;           // tiles of the recompute's shape
  Tile* d_tiles = nullptr;
  std::vector<Tile> hvtiles;          // tiles of the VJP's shape
  Tile* d_vtiles = nullptr;
  double* d_hist = nullptr;   // c_max of every stage state of a segment, 3 per state
  double* d_cpart = nullptr;
  double** d_ptrs = nullptr;
  unsigned char* d_codes = nullptr;   // reconstruction piece codes of every stage state of a segment
  long long code_plane = 0;           // bytes per direction: 8 per cell and per upper fixed-face cell
  FixedFace* d_faces = nullptr;       // the fixed faces
  int nfaces = 0;
  double* d_gadj = nullptr;           // boundary-data adjoint, nvar planes of ghost_cells
  int grid_ghost = 0;
  int grid_vjp = 0;
  int grid_emit = 0;
  int grid_small = 0;
  // overlapped recompute: the context's second stream and its events
  hipStream_t side = nullptr;
  hipEvent_t ev_fwd = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};

  ~Adj() {
    if (side) (void)hipStreamSynchronize(side);
    if (d_tiles) (void)hipFree(d_tiles);
    if (d_vtiles) (void)hipFree(d_vtiles);
    if (d_hist) (void)hipFree(d_hist);
    if (d_cpart) (void)hipFree(d_cpart);
    if (d_ptrs) (void)hipFree(d_ptrs);
    if (d_codes) (void)hipFree(d_codes);
    if (d_faces) (void)hipFree(d_faces);
    if (d_gadj) (void)hipFree(d_gadj);
  }

  int ntiles() const { return (int)htiles.size(); }
  int nvtiles() const { return (int)hvtiles.size(); }

  // dst = sum of coefficient * buffer over `terms` (launches of at most 6
  // sources; later launches carry the partial sum in dst).
  void combine(int dst, const std::vector<std::pair<int, double>>& terms) {
    size_t q = 0;
    bool first = true;
    while (q < terms.size()) {
      CombineParams p{};
      p.dst = dst;
      p.st = state_table(c);
      p.tiles = d_vtiles;
      p.ntiles = nvtiles();
      p.tx = V->tx;
      p.ty = V->ty;
      p.tz = V->tz;
      p.nv = c->nvar;
      p.n = 0;
      if (!first) {   // continue an accumulation of more than 6 terms
        p.src[p.n] = dst;
        p.a[p.n] = 1.0;
        ++p.n;
      }
      for (; q < terms.size() && p.n < 6; ++q) {
        p.src[p.n] = terms[q].first;
        p.a[p.n] = terms[q].second;
        ++p.n;
      }
      launch_combine(p, grid_small, c->stream);
      first = false;
    }
  }

  // dst = sum lam_t + dt * J_L(state)^T (sum mu_t), including the c_max
  // term; `codes` are the reconstruction pieces of L(state) and cm its c_max,
  // both from the recompute
  void vjp(int state, const unsigned char* codes, const double* cm, const std::vector<std::pair<int, double>>& mu_t,
           const std::vector<std::pair<int, double>>& lam_t, int dst, double dt) {
    StateTable st = state_table(c);
    VjpParams p{};
    p.st = st;
    p.tiles = d_vtiles;
    p.ntiles = nvtiles();
    p.ctl = c->d_ctl;
    p.gamma = c->cfg.gamma;
    p.in = state;
    p.codes = codes;
    p.code_plane = code_plane;
    p.code_faces = c->total_cells;
    p.recon = c->cfg.recon;
    p.nmu = (int)mu_t.size();
    for (int q = 0; q < p.nmu; ++q) {
      p.mu_src[q] = mu_t[q].first;
      p.mu_a[q] = mu_t[q].second;
    }
    p.nlam = (int)lam_t.size();
    for (int q = 0; q < p.nlam; ++q) {
      p.lam_src[q] = lam_t[q].first;
      p.lam_a[q] = lam_t[q].second;
    }
    p.dst = dst;
    p.scale = dt;
    p.cm_in = cm;
    p.cpart = d_cpart;
    V->launch(p, grid_vjp, c->stream);
    int nparts = grid_vjp;
    if (nfaces > 0) {   // the ghost cells of fixed faces: boundary-data adjoint, their c_max share
      V->ghost(p, d_faces, nfaces, d_gadj, c->ghost_cells, d_cpart + 3 * (size_t)grid_vjp, grid_ghost, c->stream);
      nparts += grid_ghost;
    }
    V->cmax_term(st, (int)c->hb.size(), d_cpart, nparts, c->d_ctl, c->cfg.gamma, state, dst, dt, c->stream);
  }
};

}  // namespace

extern "C" amrvac_status amrvac_ssprk_adjoint(amrvac_ctx* c, int scheme, double dt, int nsteps, int ckpt_every,
                                              double* const* lam) {
  if (!c) return AMRVAC_ERR_INVALID;
  if (c->hb.empty()) return ctx_fail(c, AMRVAC_ERR_INVALID, "ssprk_adjoint: no blocks set");
  if (!lam) return ctx_fail(c, AMRVAC_ERR_INVALID, "ssprk_adjoint: lam is NULL");
  const int nb = (int)c->hb.size();
  for (int b = 0; b < nb; ++b)
    if (!lam[b]) return ctx_fail(c, AMRVAC_ERR_INVALID, "ssprk_adjoint: lam[%d] is NULL", b);
  if (scheme < AMRVAC_RK3 || scheme > AMRVAC_SSPRK54 || nsteps < 0 || ckpt_every < 1 || !std::isfinite(dt) ||
      !(dt > 0.0))
    return ctx_fail(c, AMRVAC_ERR_INVALID, "ssprk_adjoint: invalid scheme, nsteps, ckpt_every or dt");
  if (c->n_active < nb) return ctx_fail(c, AMRVAC_ERR_UNSUPPORTED, "ssprk_adjoint: some blocks are passive");
  if (c->cfg.physics == AMRVAC_GLM) return ctx_fail(c, AMRVAC_ERR_UNSUPPORTED, "ssprk_adjoint: GLM is not supported");
  if (c->cfg.eta_h > 0.0) return ctx_fail(c, AMRVAC_ERR_UNSUPPORTED, "ssprk_adjoint: Hall MHD is not supported");
  for (int b = 0; b < nb; ++b)
    for (int d = 0; d < c->cfg.ndim; ++d) {
      if (c->hb[b].n[d] < 5)
        return ctx_fail(c, AMRVAC_ERR_UNSUPPORTED, "ssprk_adjoint: block %d has n[%d] < 5", b, d);
    }
  for (int b = 0; b < nb; ++b)
    for (int d = 0; d < c->cfg.ndim; ++d)
      for (int s = 0; s < 2; ++s)
        if (c->hb[b].nbr[2 * d + s] >= 0 && c->hb[c->hb[b].nbr[2 * d + s]].n[d] < 5)
          return ctx_fail(c, AMRVAC_ERR_UNSUPPORTED, "ssprk_adjoint: neighbour of block %d has n[%d] < 5", b, d);

  const int s = scheme_stages(scheme);
  const int N = nsteps;
  const int k = std::max(1, std::min(ckpt_every, std::max(N, 1)));
  const int M = (N + k - 1) / k;   // segments
  const VjpVariant* VV = vjp_variant(c->cfg.ndim, c->cfg.physics == AMRVAC_MHD);
  const StageVariant* EV = emit_variant(c->cfg.ndim, c->cfg.physics == AMRVAC_MHD, c->cfg.recon);
  if (!VV || !EV) return ctx_fail(c, AMRVAC_ERR_UNSUPPORTED, "ssprk_adjoint: no kernel for this ndim/physics");
  // Lists whose recompute and VJP launches hold at most two work-groups per
  // CU leave most of the GPU idle in each launch: there the next segment is
  // recomputed on a second stream (into a second set of stage states and
  // codes) while this one is reversed.  AMRVAC_ADJOINT_OVERLAP=0/1 overrides.
  bool overlap = false;
  {
    long long tv = 0, te = 0;
    for (int b = 0; b < nb; ++b) {
      long long a = 1, e = 1;
      const int TV[3] = {VV->tx, VV->ty, VV->tz}, TE[3] = {EV->tx, EV->ty, EV->tz};
      for (int d = 0; d < 3; ++d) {
        a *= (c->hb[b].n[d] + TV[d] - 1) / TV[d];
        e *= (c->hb[b].n[d] + TE[d] - 1) / TE[d];
      }
      tv += a;
      te += e;
    }
    overlap = M > 1 && tv <= 2LL * c->ncu && te <= 2LL * c->ncu;
    const char* env = std::getenv("AMRVAC_ADJOINT_OVERLAP");
    if (env && *env) overlap = M > 1 && env[0] == '1';
  }
  const int sets = overlap ? 2 : 1;
  // buffer ids (scratch slot = id - 1)
  const int A = 1, Bf = 2, W1 = 5;
  int Sset[2] = {3, 0}, W0set[2] = {4, 0};
  int next = 6;
  std::vector<int> ck(std::max(M, 1), 0);   // ck[0] = caller's U0 (id 0)
  for (int m = 1; m < M; ++m) ck[m] = next++;
  // stage states of a segment, per set: X[set][j][i] (X[set][j][0] of j = 0
  // is the segment's checkpoint)
  std::vector<std::vector<std::vector<int>>> X(sets, std::vector<std::vector<int>>(k, std::vector<int>(s, 0)));
  for (int set = 0; set < sets; ++set) {
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < s; ++i) X[set][j][i] = next++;
    if (set > 0) {
      Sset[set] = next++;
      W0set[set] = next++;
    }
  }
  const int S = Sset[0], W0 = W0set[0];
  std::vector<int> Lm(s + 1);
  for (int i = 0; i <= s; ++i) Lm[i] = next++;
  // memory: state slots (the context keeps them for later calls) and the
  // piece codes of one segment (freed on return); both grow with the
  // checkpoint interval k, as (5 + segments + k s + s) slots and k s ndim
  // code planes.  Refuse up front, with the figures, what cannot fit.
  {
    long long fw = 0;
    for (int d = 0; d < 3; ++d) fw = std::max(fw, c->face_words[d]);
    const double slot_bytes = 8.0 * (double)c->slot_stride;
    const double grow = next - 1 > c->nslots ? slot_bytes * (double)(next - 1 - c->nslots) : 0.0;
    const double codes = 8.0 * (double)(c->total_cells + fw) * c->cfg.ndim * s * (double)k * sets;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && grow + codes > 0.97 * (double)free_b)
      return ctx_fail(c, AMRVAC_ERR_NOMEM,
                      "ssprk_adjoint: checkpoints every %d steps need %.1f GB more device memory (%d state slots, "
                      "%.1f GB of piece codes) than the %.1f GB free; use a smaller ckpt_every",
                      k, (grow + codes) / 1e9, next - 1, codes / 1e9, (double)free_b / 1e9);
  }
  amrvac_status st = ensure_slots(c, next - 1);
  if (st != AMRVAC_OK) return st;

  Adj adj;
  adj.c = c;
  adj.V = VV;
  // one tile list per shape: the recompute's and the VJP's
  for (int which = 0; which < 2; ++which) {
    const int T[3] = {which ? adj.V->tx : EV->tx, which ? adj.V->ty : EV->ty, which ? adj.V->tz : EV->tz};
    std::vector<Tile>& out = which ? adj.hvtiles : adj.htiles;
    for (int b = 0; b < nb; ++b) {
      const amrvac_block& q = c->hb[b];
      int nt[3];
      for (int d = 0; d < 3; ++d) nt[d] = (q.n[d] + T[d] - 1) / T[d];
      for (int z = 0; z < nt[2]; ++z)
        for (int y = 0; y < nt[1]; ++y)
          for (int x = 0; x < nt[0]; ++x) {
            Tile t;
            t.block = b;
            t.o[0] = x * T[0];
            t.o[1] = y * T[1];
            t.o[2] = z * T[2];
            out.push_back(t);
          }
    }
  }
  const int nt = adj.ntiles();
  auto hip_ok = [&](hipError_t e, const char* what) -> amrvac_status {
    if (e == hipSuccess) return AMRVAC_OK;
    return ctx_fail(c, e == hipErrorOutOfMemory ? AMRVAC_ERR_NOMEM : AMRVAC_ERR_DEVICE, "%s: %s", what,
                    hipGetErrorString(e));
  };
  const int nvt = adj.nvtiles();
  if ((st = hip_ok(hipMalloc(&adj.d_tiles, sizeof(Tile) * nt), "hipMalloc")) != AMRVAC_OK) return st;
  if ((st = hip_ok(hipMalloc(&adj.d_vtiles, sizeof(Tile) * nvt), "hipMalloc")) != AMRVAC_OK) return st;
  if ((st = hip_ok(hipMalloc(&adj.d_hist, sizeof(double) * 3 * (size_t)s * (size_t)k * sets), "hipMalloc")) !=
      AMRVAC_OK)
    return st;
  // the maximiser keys start above every valid key (the VJPs lower them)
  if ((st = hip_ok(hipMemsetAsync(c->d_ctl->arg, 0x7f, sizeof(c->d_ctl->arg), c->stream), "memset")) != AMRVAC_OK)
    return st;
  std::vector<FixedFace> hfaces;
  for (int b = 0; b < nb; ++b)
    for (int f = 0; f < 2 * c->cfg.ndim; ++f)
      if (c->hb[b].nbr[f] < 0) hfaces.push_back(FixedFace{b, f});
  adj.nfaces = (int)hfaces.size();
  adj.grid_ghost = std::max(1, std::min(adj.nfaces, c->ncu * 4));
  if ((st = hip_ok(hipMalloc(&adj.d_cpart, sizeof(double) * 3 * ((size_t)nvt + adj.grid_ghost)), "hipMalloc")) !=
      AMRVAC_OK)
    return st;
  if (adj.nfaces > 0) {
    if ((st = hip_ok(hipMalloc(&adj.d_faces, sizeof(FixedFace) * hfaces.size()), "hipMalloc")) != AMRVAC_OK) return st;
    if ((st = hip_ok(hipMemcpyAsync(adj.d_faces, hfaces.data(), sizeof(FixedFace) * hfaces.size(),
                                    hipMemcpyHostToDevice, c->stream), "upload")) != AMRVAC_OK)
      return st;
    const size_t gbytes = sizeof(double) * (size_t)c->nvar * (size_t)c->ghost_cells;
    if ((st = hip_ok(hipMalloc(&adj.d_gadj, gbytes), "hipMalloc")) != AMRVAC_OK) return st;
    if ((st = hip_ok(hipMemsetAsync(adj.d_gadj, 0, gbytes, c->stream), "memset")) != AMRVAC_OK) return st;
  }
  if ((st = hip_ok(hipMalloc(&adj.d_ptrs, sizeof(double*) * nb), "hipMalloc")) != AMRVAC_OK) return st;
  if ((st = hip_ok(hipMemcpyAsync(adj.d_tiles, adj.htiles.data(), sizeof(Tile) * nt, hipMemcpyHostToDevice,
                                  c->stream), "upload")) != AMRVAC_OK)
    return st;
  if ((st = hip_ok(hipMemcpyAsync(adj.d_vtiles, adj.hvtiles.data(), sizeof(Tile) * nvt, hipMemcpyHostToDevice,
                                  c->stream), "upload")) != AMRVAC_OK)
    return st;
  std::vector<double*> hptrs(lam, lam + nb);
  if ((st = hip_ok(hipMemcpyAsync(adj.d_ptrs, hptrs.data(), sizeof(double*) * nb, hipMemcpyHostToDevice, c->stream),
                   "upload")) != AMRVAC_OK)
    return st;
  // codes of the k * s stage states of one segment, ndim planes each
  long long fw = 0;
  for (int d = 0; d < 3; ++d) fw = std::max(fw, c->face_words[d]);
  adj.code_plane = (c->total_cells + fw) * 8;
  const size_t code_bytes = (size_t)adj.code_plane * (size_t)c->cfg.ndim * (size_t)s * (size_t)k * sets;
  if ((st = hip_ok(hipMalloc(&adj.d_codes, code_bytes), "hipMalloc (MP5 piece codes)")) != AMRVAC_OK) return st;
  auto codes_of = [&](int set, int j, int kst) {
    return adj.d_codes + (((size_t)set * k + j) * s + kst) * (size_t)c->cfg.ndim * (size_t)adj.code_plane;
  };
  auto hist_of = [&](int set, int j, int kst) { return adj.d_hist + 3 * (((size_t)set * k + j) * s + kst); };
  if (overlap) {
    if (!c->adj_side &&
        (st = hip_ok(hipStreamCreateWithFlags(&c->adj_side, hipStreamNonBlocking), "stream")) != AMRVAC_OK)
      return st;
    for (hipEvent_t& e : c->adj_ev)
      if (!e && (st = hip_ok(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event")) != AMRVAC_OK) return st;
    adj.side = c->adj_side;
    adj.ev_fwd = c->adj_ev[0];
    adj.ev_rec[0] = c->adj_ev[1];
    adj.ev_rec[1] = c->adj_ev[2];
    adj.ev_rev[0] = c->adj_ev[3];
    adj.ev_rev[1] = c->adj_ev[4];
  }
  int per_cu = 0;
  if ((st = hip_ok(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, adj.V->fn, adj.V->nt, 0), "occupancy")) !=
      AMRVAC_OK)
    return st;
  adj.grid_vjp = std::max(1, std::min(std::max(per_cu, 1) * c->ncu, nvt));
  per_cu = 0;
  if ((st = hip_ok(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, EV->fn, EV->nt, 0), "occupancy")) !=
      AMRVAC_OK)
    return st;
  adj.grid_emit = std::max(1, std::min(std::max(per_cu, 1) * c->ncu, nt));
  adj.grid_small = std::max(1, std::min(c->ncu * 8, nvt));

  double alpha[6][6], beta[6][6];
  scheme_table(scheme, alpha, beta);
  const int exec = AMRVAC_EXEC_BATCHED;

  // ---- forward pass to the checkpoints (U0 = caller's u, read only) ----
  launch_set_control(c->d_ctl, dt, 0.4, 0.0, c->stream);
  int cur = 0;
  const int last_needed = (M - 1) * k;   // states beyond the last checkpoint are not needed
  if (last_needed > 0) launch_cmax_of(c, cur, 0, c->stream);
  for (int n = 0; n < last_needed; ++n) {
    int nxt;
    if ((n + 1) % k == 0) {
      nxt = ck[(n + 1) / k];
    } else {
      nxt = (cur == W0) ? W1 : W0;
    }
    int outs[6];
    for (int i = 1; i <= s; ++i) outs[i] = (i == s) ? nxt : ((i % 2) ? A : Bf);
    enqueue_step_outs(c, scheme, exec, c->stream, cur, outs, S);
    cur = nxt;
  }

  // ---- reverse sweep over segments ----
  int R = Lm[s];   // running adjoint of the current output state
  launch_lam_import(state_table(c), adj.d_ptrs, c->nvar, R, nb, c->stream);
  std::vector<int> lslots(Lm.begin(), Lm.end());
  // recompute segment m into stage-state set `set`, storing every stage state
  auto recompute = [&](int m, int set, hipStream_t strm) {
    const int kk = std::min(k, N - m * k);
    std::vector<std::vector<int>>& XX = X[set];
    XX[0][0] = ck[m];
    launch_cmax_of(c, XX[0][0], 0, strm);
    for (int j = 0; j < kk; ++j) {
      int outs[6];
      for (int i = 1; i < s; ++i) outs[i] = XX[j][i];
      outs[s] = (j + 1 < kk) ? XX[j + 1][0] : W0set[set];   // the segment's last output is not needed
      EmitPlan plan{};
      plan.var = EV;
      plan.tiles = adj.d_tiles;
      plan.ntiles = nt;
      plan.grid = adj.grid_emit;
      for (int i = 0; i < s; ++i) {
        plan.codes[i] = codes_of(set, j, i);
        plan.cm_hist[i] = hist_of(set, j, i);
      }
      plan.code_plane = adj.code_plane;
      enqueue_step_outs(c, scheme, exec, strm, XX[j][0], outs, Sset[set], &plan);
    }
  };
  // reverse segment m's steps from stage-state set `set` (context stream)
  auto reverse = [&](int m, int set) {
    const int kk = std::min(k, N - m * k);
    for (int j = kk - 1; j >= 0; --j) {
      // lam(s) = R; lam(i) for i < s are the other slots
      std::vector<int> L(s + 1);
      L[s] = R;
      {
        int q = 0;
        for (int id : lslots)
          if (id != R && q < s) L[q++] = id;
      }
      for (int kst = s - 1; kst >= 0; --kst) {
        std::vector<std::pair<int, double>> mu_t, lam_t;
        for (int i = kst + 1; i <= s; ++i) {
          if (beta[i][kst] != 0.0) mu_t.push_back({L[i], beta[i][kst]});
          if (alpha[i][kst] != 0.0) lam_t.push_back({L[i], alpha[i][kst]});
        }
        if (lam_t.empty()) lam_t.push_back({L[s], 0.0});
        if (mu_t.empty())
          adj.combine(L[kst], lam_t);
        else
          adj.vjp(X[set][j][kst], codes_of(set, j, kst), hist_of(set, j, kst), mu_t, lam_t, L[kst], dt);
      }
      R = L[0];
    }
  };
  if (!overlap) {
    for (int m = M - 1; m >= 0; --m) {
      recompute(m, 0, c->stream);
      reverse(m, 0);
    }
  } else {
    // the second stream starts after the forward pass; segment m uses set
    // m % 2, whose previous user (segment m + 2) must be reversed first
    hipError_t err = hipSuccess;
    auto ok = [&](hipError_t e) {
      if (e != hipSuccess && err == hipSuccess) err = e;
      return err == hipSuccess;
    };
    if (ok(hipEventRecord(adj.ev_fwd, c->stream)) && ok(hipStreamWaitEvent(adj.side, adj.ev_fwd, 0))) {
      recompute(M - 1, (M - 1) % 2, adj.side);
      ok(hipEventRecord(adj.ev_rec[(M - 1) % 2], adj.side));
    }
    for (int m = M - 1; m >= 0 && err == hipSuccess; --m) {
      const int set = m % 2;
      if (!ok(hipStreamWaitEvent(c->stream, adj.ev_rec[set], 0))) break;
      if (m >= 1) {
        if (m + 1 <= M - 1 && !ok(hipStreamWaitEvent(adj.side, adj.ev_rev[1 - set], 0))) break;
        recompute(m - 1, 1 - set, adj.side);
        if (!ok(hipEventRecord(adj.ev_rec[1 - set], adj.side))) break;
      }
      reverse(m, set);
      ok(hipEventRecord(adj.ev_rev[set], c->stream));
    }
    if (err != hipSuccess) return hip_ok(err, "adjoint streams");
  }
  launch_lam_export(state_table(c), adj.d_ptrs, c->nvar, R, nb, adj.d_gadj, c->ghost_cells, c->stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_ok(e, "adjoint launch");
  return read_status(c);
}
