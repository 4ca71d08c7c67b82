// Host-only paths of the C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_sanitizers.py): block-list
// validation and the activation safety belt, on valid and invalid inputs.
// No device is touched.  The kernel-side entry points the runtime links
// against are stubbed: none of the paths exercised here reaches them.
#include <cstdio>
#include <cstring>
#include <vector>

#include "amrvac.h"
#include "runtime_internal.h"

namespace amrvac {
const StageVariant* stage_variants(int* count) {
  *count = 0;
  return nullptr;
}
const StageVariant* emit_variant(int, int, int) { return nullptr; }
void launch_cmax(int, int, const CmaxParams&, int, hipStream_t) {}
void launch_current(int, const StateTable&, const Tile*, int, int, int, int, int, double*, long long, int,
                    hipStream_t) {}
void launch_divb(int, const StateTable&, const Tile*, int, int, int, int, int, double* const*, double*, double*,
                 int, hipStream_t) {}
void launch_step_begin(Control*, const double*, int, int, int, int, hipStream_t) {}
void launch_clear_slot(Control*, int, hipStream_t) {}
void launch_set_control(Control*, double, double, double, hipStream_t) {}
void launch_copy_interior(const StateTable&, const Tile*, int, int, int, int, int, int, int, int, hipStream_t) {}
}  // namespace amrvac

static int failures = 0;
#define CHECK(cond)                                                  \
  do {                                                               \
    if (!(cond)) {                                                   \
      std::fprintf(stderr, "CHECK failed line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                    \
    }                                                                \
  } while (0)

// A periodic nx x ny grid of blocks of m x m cells (2D).
static std::vector<amrvac_block> grid2d(int nx, int ny, int m, std::vector<double>& storage) {
  std::vector<amrvac_block> b(nx * ny);
  storage.assign(16, 0.0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      amrvac_block& q = b[j * nx + i];
      std::memset(&q, 0, sizeof(q));
      q.u = storage.data();
      q.n[0] = q.n[1] = m;
      q.n[2] = 1;
      q.dx[0] = q.dx[1] = 1.0 / (m * nx);
      q.dx[2] = 1.0;
      q.nbr[0] = j * nx + (i + nx - 1) % nx;
      q.nbr[1] = j * nx + (i + 1) % nx;
      q.nbr[2] = ((j + ny - 1) % ny) * nx + i;
      q.nbr[3] = ((j + 1) % ny) * nx + i;
      q.nbr[4] = q.nbr[5] = -1;
    }
  return b;
}

int main() {
  amrvac_config cfg;
  std::memset(&cfg, 0, sizeof(cfg));
  cfg.ndim = 2;
  cfg.physics = AMRVAC_HD;
  cfg.gamma = 1.4;
  cfg.exec = AMRVAC_EXEC_BATCHED;
  cfg.recon = AMRVAC_MP5;
  char msg[256];
  std::vector<double> st;
  std::vector<amrvac_block> g = grid2d(3, 2, 8, st);
  CHECK(amrvac_validate_blocks(&cfg, g.data(), (int)g.size(), msg, sizeof(msg)) == AMRVAC_OK);
  // every kind of invalid list, and a tiny message buffer
  std::vector<amrvac_block> bad = g;
  bad[1].nbr[0] = 5;   // not symmetric
  CHECK(amrvac_validate_blocks(&cfg, bad.data(), (int)bad.size(), msg, sizeof(msg)) == AMRVAC_ERR_INVALID);
  CHECK(amrvac_validate_blocks(&cfg, bad.data(), (int)bad.size(), msg, 1) == AMRVAC_ERR_INVALID);
  bad = g;
  bad[2].nbr[3] = 99;  // out of range
  CHECK(amrvac_validate_blocks(&cfg, bad.data(), (int)bad.size(), msg, sizeof(msg)) == AMRVAC_ERR_INVALID);
  bad = g;
  bad[0].n[0] = 2;     // fewer than 3 cells
  CHECK(amrvac_validate_blocks(&cfg, bad.data(), (int)bad.size(), msg, sizeof(msg)) == AMRVAC_ERR_INVALID);
  bad = g;
  bad[4].u = nullptr;
  CHECK(amrvac_validate_blocks(&cfg, bad.data(), (int)bad.size(), msg, sizeof(msg)) == AMRVAC_ERR_INVALID);
  bad = g;
  bad[3].dx[1] = -1.0;
  CHECK(amrvac_validate_blocks(&cfg, bad.data(), (int)bad.size(), msg, sizeof(msg)) == AMRVAC_ERR_INVALID);
  bad = g;
  bad[3].n[2] = 2;     // inactive direction must have one cell
  CHECK(amrvac_validate_blocks(&cfg, bad.data(), (int)bad.size(), msg, sizeof(msg)) == AMRVAC_ERR_INVALID);
  CHECK(amrvac_validate_blocks(&cfg, nullptr, 3, msg, sizeof(msg)) == AMRVAC_ERR_INVALID);
  CHECK(amrvac_validate_blocks(&cfg, g.data(), 0, nullptr, 0) == AMRVAC_ERR_INVALID);
  CHECK(amrvac_validate_blocks(nullptr, g.data(), (int)g.size(), msg, sizeof(msg)) == AMRVAC_ERR_INVALID);
  amrvac_config c2 = cfg;
  c2.gamma = 1.0;
  CHECK(amrvac_validate_blocks(&c2, g.data(), (int)g.size(), msg, sizeof(msg)) == AMRVAC_ERR_INVALID);
  c2 = cfg;
  c2.eta_h = 0.1;      // Hall needs MHD
  CHECK(amrvac_validate_blocks(&c2, g.data(), (int)g.size(), msg, sizeof(msg)) == AMRVAC_ERR_INVALID);

  // activation flags: safety belt on the periodic 3 x 2 grid
  const int nb = (int)g.size();
  std::vector<unsigned char> want(nb, 0), out(nb, 7);
  want[0] = 1;
  CHECK(amrvac_activation_flags(g.data(), nb, want.data(), 0, out.data()) == 1);
  CHECK(amrvac_activation_flags(g.data(), nb, want.data(), 1, out.data()) == 4);
  CHECK(amrvac_activation_flags(g.data(), nb, want.data(), 5, out.data()) == nb);
  CHECK(amrvac_activation_flags(nullptr, nb, want.data(), 1, out.data()) == -1);
  CHECK(amrvac_activation_flags(g.data(), nb, nullptr, 1, out.data()) == -1);
  CHECK(amrvac_activation_flags(g.data(), nb, want.data(), -1, out.data()) == -1);
  CHECK(amrvac_activation_flags(g.data(), 0, want.data(), 1, out.data()) == -1);
  bad = g;
  bad[2].nbr[1] = -7;
  CHECK(amrvac_activation_flags(bad.data(), nb, want.data(), 1, out.data()) == -1);
  // a single block, periodic onto itself, and a long chain of fixed faces
  std::vector<amrvac_block> one = grid2d(1, 1, 5, st);
  std::vector<unsigned char> w1(1, 1), o1(1, 0);
  CHECK(amrvac_activation_flags(one.data(), 1, w1.data(), 3, o1.data()) == 1);
  std::vector<amrvac_block> chain = grid2d(64, 1, 4, st);
  for (auto& q : chain) q.nbr[2] = q.nbr[3] = -1;
  chain.front().nbr[0] = -1;
  chain.back().nbr[1] = -1;
  std::vector<unsigned char> wc(64, 0), oc(64, 0);
  wc[10] = 1;
  CHECK(amrvac_activation_flags(chain.data(), 64, wc.data(), 3, oc.data()) == 7);
  CHECK(oc[7] == 1 && oc[13] == 1 && oc[6] == 0 && oc[14] == 0);
  cfg.ndim = 1;
  for (auto& q : chain) q.n[1] = 1, q.dx[1] = 1.0, q.nbr[2] = q.nbr[3] = -1;
  CHECK(amrvac_validate_blocks(&cfg, chain.data(), 64, msg, sizeof(msg)) == AMRVAC_OK);
  std::printf("host paths: %d failure(s)\n", failures);
  return failures == 0 ? 0 : 1;
}
