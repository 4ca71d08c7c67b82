// Reverse mode of the SSPRK time integration (amrvac_ssprk_adjoint).
#include "amrvac.h"
#include "amrvac_internal.h"

#include <cmath>
#include <vector>

namespace amrvac {
amrvac_status ctx_fail(amrvac_ctx* c, amrvac_status st, const char* msg);
}
using namespace amrvac;

extern "C" amrvac_status amrvac_ssprk_adjoint(amrvac_ctx* c, int scheme, double dt, int nsteps,
                                              int ckpt_every, double* const* lam) {
  if (!c) return AMRVAC_ERR_INVALID;
  if (!lam) return ctx_fail(c, AMRVAC_ERR_INVALID, "ssprk_adjoint: lam is NULL");
  if (scheme < AMRVAC_RK3 || scheme > AMRVAC_SSPRK54 || nsteps < 0 || ckpt_every < 1 ||
      !std::isfinite(dt) || !(dt > 0.0))
    return ctx_fail(c, AMRVAC_ERR_INVALID, "ssprk_adjoint: invalid scheme, nsteps, ckpt_every or dt");
  return ctx_fail(c, AMRVAC_ERR_UNSUPPORTED, "ssprk_adjoint: not available in this build");
}
