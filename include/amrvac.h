/*
 * amrvac.h -- C ABI of the MI355X (gfx950) FP64 hot path of the conservative
 * high-order finite-difference scheme of Porth et al. (2014), "MPI-AMRVAC for
 * Solar and Astrophysics", Sect. 2:
 *
 *   dU/dt = L(U) = - sum_d (Fhat_{d,i+1/2} - Fhat_{d,i-1/2}) / dx_d
 *     (Sect. 2.1, eqs. fdcons, reconstruct, timeoperator; no source terms),
 *   Fhat = R_[L](F^+) + R_[R](F^-),  F^+- = (F +- c_max U) / 2
 *     (Sect. 2.2, global Lax-Friedrichs flux-vector splitting),
 *   R = MP5 (Suresh & Huynh 1997) or LIM03 (Cada & Torrilhon 2009), the two
 *     reconstructions Sect. 2.2 offers for the FD scheme,
 *   U^(i) = sum_k alpha_ik U^(k) + dt beta_ik L(U^(k))
 *     (Sect. 2.3, Shu-Osher form; RK3, SSPRK(4,3), SSPRK(5,4)),
 *
 * for ideal hydrodynamics (Sect. 3, ideal-gas energy equation), ideal MHD
 * (Sects. 4.1 and 4.3 with B0 = 0, eta = eta_h = 0), GLM-MHD (Sect. 4.2, the
 * glm3 variant) and Hall MHD (Sect. 4.4, eta_h > 0, eta = 0).
 *
 * Conventions shared by every call
 * --------------------------------
 *  * All floating point is IEEE binary64.
 *  * A "block" is a Cartesian box of n[0] x n[1] x n[2] interior cells
 *    (n[d] = 1 for d >= ndim) stored with AMRVAC_NGHOST = 3 ghost layers on
 *    both sides of every active direction: nvar arrays of
 *    P0 * P1 * P2 doubles (P_d = n[d] + 6 if d < ndim, else 1), variable
 *    major, x fastest.  Variables: hydro (rho, m_1..m_ndim, E), nvar =
 *    2 + ndim; MHD (rho, m_x, m_y, m_z, E, B_x, B_y, B_z), nvar = 8; GLM as
 *    MHD followed by psi, nvar = 9.  Values are point values at cell centres
 *    (Sect. 2.1).
 *  * Faces: nbr[2d] (low side) and nbr[2d+1] (high side) of direction d are
 *    either the index of the neighbouring block in the list (its interior
 *    supplies the 3 ghost layers; periodic wrap is expressed by the caller
 *    through these indices) or -1, meaning the ghost layers of this block
 *    hold caller-filled boundary values that stay constant in time.  Only
 *    face ghosts are read (the operator is a sum of 1D stencils); edge and
 *    corner ghosts are never read.  Periodic ghost layers are neither read
 *    nor written.
 *  * c_max (Sect. 2.2) is the maximum over all interior cells of all blocks
 *    of |v_d| + c_f,d, per direction d, of the state L is applied to (c_f:
 *    fast magnetosonic speed along d; the sound speed for hydro).
 *  * Device pointers are HIP device addresses; the caller owns them.  Every
 *    call is stream-ordered on the stream given to amrvac_create and does
 *    not synchronise the host unless stated.
 *  * Errors: a call returns a status.  Host-detectable errors (null
 *    pointers, bad sizes, inconsistent neighbours, unsupported options) are
 *    reported before anything is enqueued, leaving all state unchanged.
 *    Device-detected errors (rho <= 0, p <= 0 or a non-finite value met by
 *    the primitive recovery) set a sticky flag that the next synchronising
 *    call (amrvac_sync, or a call documented to synchronise) returns as
 *    AMRVAC_ERR_NONPHYSICAL; the state is then unspecified.  No call aborts
 *    or throws across the ABI.
 *  * A context is used from one host thread at a time.
 */
#ifndef AMRVAC_H
#define AMRVAC_H

#ifdef __cplusplus
extern "C" {
#endif

#define AMRVAC_ABI_VERSION 5
#define AMRVAC_NGHOST 3

typedef enum {
  AMRVAC_OK = 0,
  AMRVAC_ERR_INVALID = 1,      /* bad argument, layout or neighbour table      */
  AMRVAC_ERR_NOMEM = 2,        /* device allocation failed                     */
  AMRVAC_ERR_DEVICE = 3,       /* HIP runtime error                            */
  AMRVAC_ERR_NONPHYSICAL = 4,  /* rho <= 0, p <= 0 or non-finite state met     */
  AMRVAC_ERR_UNSUPPORTED = 5   /* valid request this build does not implement  */
} amrvac_status;

/* GLM (Sect. 4.2, glm3): psi is added to the flux of B_d and c_h^2 B_d is
 * the flux of psi along d; no other psi or div B terms.  The cleaning speed
 * c_h is the largest per-direction c_max of the state a right-hand side is
 * evaluated on, and every direction then uses c_h in place of its c_max (in
 * the Lax-Friedrichs split, the time step, and the cmax_out of
 * amrvac_fd_rhs).  After each time step psi is multiplied by
 * exp(-dt c_h / c_r), c_h of the step's initial state, c_r = c_p^2 / c_h =
 * 0.18 (operator split).  amrvac_ssprk_adjoint does not support GLM
 * (AMRVAC_ERR_UNSUPPORTED). */
typedef enum { AMRVAC_HD = 0, AMRVAC_MHD = 1, AMRVAC_GLM = 2 } amrvac_physics;

/* Sect. 2.3: RK3 (Gottlieb & Shu 1998), SSPRK(4,3) and SSPRK(5,4) tables. */
typedef enum { AMRVAC_RK3 = 0, AMRVAC_SSPRK43 = 1, AMRVAC_SSPRK54 = 2 } amrvac_scheme;

/* Execution form of a stage (every form gives bitwise the same result):
 *  PER_BLOCK:       one launch per block and stage;
 *  BATCHED:         persistent fused launches over the block list, one per
 *                   block-size class (blocks of equal cell count; a class
 *                   with fewer tiles than twice the resident work-groups
 *                   joins the next), steps replayed from HIP graphs (of 8
 *                   steps, and of one step for the remainder of a call);
 *  BATCHED_SINGLE:  one persistent fused launch per stage over the whole
 *                   list (each XCD's share holds an eighth of every class),
 *                   steps replayed from HIP graphs as for BATCHED.
 * Setting a batched form rebuilds the work list; the autotuner times tile
 * shapes in the form that is set. */
typedef enum { AMRVAC_EXEC_PER_BLOCK = 0, AMRVAC_EXEC_BATCHED = 1, AMRVAC_EXEC_BATCHED_SINGLE = 2 } amrvac_exec;

/* Reconstruction of the split fluxes (Sect. 2.2).
 *  MP5:   Suresh & Huynh (1997) with alpha = 4 and eps = 0; 5-cell stencils,
 *         reads all 3 ghost layers.
 *  LIM03: Cada & Torrilhon (2009) compact third-order function with the
 *         asymptotic-region switch: from f_{j-1}, f_j, f_{j+1}, with
 *         dm = f_j - f_{j-1} and dp = f_{j+1} - f_j, the interface value is
 *         f_j + H/2 with H = (2 dp + dm)/3 where (dm^2 + dp^2) <= (r dx)^2,
 *         else H = phi(dm/dp) dp, phi(t) = max(0, min(phi3, max(-t/2,
 *         min(2t, phi3, 1.6)))), phi3 = (2 + t)/3 (H = 0 for dp = 0); radius
 *         r = 1 (data units per cell width dx along the pencil).  3-cell
 *         stencils: only the 2 inner ghost layers are read. */
typedef enum { AMRVAC_MP5 = 0, AMRVAC_LIM03 = 1 } amrvac_recon;

typedef struct {
  int ndim;        /* 1, 2 or 3                                     */
  int physics;     /* amrvac_physics                                */
  double gamma;    /* ratio of specific heats, finite and > 1       */
  int exec;        /* amrvac_exec                                   */
  int recon;       /* amrvac_recon (added in ABI version 2)         */
  double eta_h;    /* Hall parameter (ABI version 3): 0 = ideal MHD;
                      > 0 only with AMRVAC_MHD, see below            */
} amrvac_config;

/* Hall MHD (Sect. 4.4, conservative Hall MHD in finite differences, eta = 0,
 * B0 = 0), selected by eta_h > 0 with AMRVAC_MHD:
 *  * before every evaluation of L the cell-centred current J = curl B is
 *    computed at every interior cell by fourth-order central differences
 *    along each active direction, (-B[i+2] + 8 B[i+1] - 8 B[i-1] + B[i-2]) /
 *    (12 dx); halo cells use their face neighbour's J, so every face of
 *    every block must have a neighbour (set_blocks refuses fixed faces);
 *  * the flux of B gains (eta_h/rho)(B_d J - J_d B) and that of E gains
 *    (eta_h/rho)((J.B) B_d - B^2 J_d);
 *  * the speed of every cell along d is |v_d| + max(c_f,d, eta_h |B| k_max /
 *    rho) with k_max = pi max_d 1/dx_d of the cell's block, in c_max (split
 *    and time step, which then scales with dx^2);
 *  * amrvac_ssprk_adjoint refuses it (AMRVAC_ERR_UNSUPPORTED). */

typedef struct {
  double *u;       /* device; padded conserved state (layout above)     */
  int n[3];        /* interior cells per direction (1 for d >= ndim)    */
  double dx[3];    /* cell widths, > 0 for active directions            */
  double xlo[3];   /* lower face of the first interior cell             */
  int nbr[6];      /* face neighbours (-x,+x,-y,+y,-z,+z) or -1 (fixed) */
} amrvac_block;

typedef struct amrvac_ctx amrvac_ctx;

/* Returns AMRVAC_ABI_VERSION. */
int amrvac_abi_version(void);

/* Creates a context on the current HIP device.  hip_stream: a hipStream_t
 * (NULL = the default stream) on which all later work is enqueued; it is
 * borrowed, not owned.  *out receives the context (NULL on failure).
 * Errors: INVALID (null cfg/out, ndim not in 1..3, physics or exec unknown,
 * gamma not finite or <= 1), DEVICE, NOMEM. */
amrvac_status amrvac_create(const amrvac_config *cfg, void *hip_stream, amrvac_ctx **out);

/* Sets the block list (Sect. 2.1 grid of point values; block/ghost layout
 * above).  The descriptors are copied; the u pointers are borrowed until the
 * next set_blocks or destroy and must stay valid and unaliased.  Builds the
 * neighbour and work tables and the context-owned scratch (stage buffers,
 * checkpoints are allocated on demand), and drops cached graphs.  Enqueues
 * table uploads on the context stream.
 * Errors: INVALID (null pointers, nblocks < 1, n[d] < 3 for an active
 * direction, n[d] != 1 or nbr != -1 for an inactive one, dx <= 0 or not
 * finite, a neighbour index out of range, a neighbour relation that is not
 * mutual (b's +d neighbour must name b as its -d neighbour), or neighbouring
 * faces of different size); NOMEM; DEVICE. */
amrvac_status amrvac_set_blocks(amrvac_ctx *ctx, const amrvac_block *blocks, int nblocks);

/* Host-only check of a block list against cfg, with the same rules as
 * amrvac_set_blocks (Sect. 2.1 grid of ghost-padded blocks).  Makes no HIP
 * call and needs no device.  msg (may be NULL) receives a description of
 * the first violation, truncated to msglen bytes including the NUL.
 * Returns OK or INVALID. */
amrvac_status amrvac_validate_blocks(const amrvac_config *cfg, const amrvac_block *blocks,
                                     int nblocks, char *msg, int msglen);

/* Chooses the execution form used by later calls (amrvac_exec). */
amrvac_status amrvac_set_exec(amrvac_ctx *ctx, int exec);

/* Tile shapes (work decomposition of the fused stage kernel) compiled for
 * this context's (ndim, physics): their number, the name of shape i (a
 * static string, NULL if i is out of range), and explicit selection of
 * shape i for later calls (rebuilds the work list and drops cached graphs;
 * results are bitwise identical for every shape).  Errors: INVALID. */
int amrvac_num_variants(const amrvac_ctx *ctx);
const char *amrvac_variant_name(const amrvac_ctx *ctx, int i);
amrvac_status amrvac_set_variant(amrvac_ctx *ctx, int i);
int amrvac_get_variant(const amrvac_ctx *ctx);   /* index in use, -1 for NULL ctx */

/* Autotuner: times nsteps steps of `scheme` (CFL 0.4) with every compiled
 * tile shape on the current block list, on scratch copies of the states
 * (the caller's buffers are only read), and keeps the fastest.  If the
 * environment variable AMRVAC_TUNE_CACHE names a file, a previous choice
 * for the same (device, ndim, physics, block count, cell count, scheme) is
 * reused without timing and new choices are appended.  ms_out (host, may
 * be NULL, amrvac_num_variants entries) receives the milliseconds per step
 * of each shape (-1 if not timed).  Synchronises the stream.
 * Errors: INVALID (no blocks, scheme unknown, nsteps < 1), NONPHYSICAL,
 * NOMEM, DEVICE. */
amrvac_status amrvac_autotune(amrvac_ctx *ctx, int scheme, int nsteps, double *ms_out);

/* Evaluates L(U) (Sect. 2.1 eq. timeoperator with S = 0, fluxes from
 * Sect. 2.2) of the current block states.  rhs: host array of nblocks
 * device pointers, each to nvar x n[0]*n[1]*n[2] doubles (interior only,
 * variable major, x fastest), written by the call.  cmax_out: host array of
 * 3 doubles receiving c_max per direction (0 for inactive ones), or NULL;
 * when non-NULL the call synchronises the context stream and reports
 * device errors.  Errors: INVALID (no blocks, null rhs or null entry),
 * NONPHYSICAL (only when synchronising), DEVICE. */
amrvac_status amrvac_fd_rhs(amrvac_ctx *ctx, double *const *rhs, double *cmax_out);

/* Divergence of B, the monitor of Sect. 4.5.1 (MHD and GLM contexts only):
 * at every interior cell of the active blocks,
 *   div B = sum over active d of (8 (B_d[i+1] - B_d[i-1]) - (B_d[i+2] -
 *           B_d[i-2])) / (12 dx_d),
 * fourth-order central differences of the blocks' state u, with the face
 * neighbours' interiors (or the fixed ghost layers) as halo.
 *  out:          NULL, or per block a device pointer to n[0]*n[1]*n[2]
 *                doubles (interior-only layout, x fastest), caller-owned;
 *  mean_abs_out: NULL, or host: the mean of |div B| over those cells, summed
 *                in a fixed order (the same bits on every call for the same
 *                state and tile shape); when non-NULL the call synchronises.
 * Errors: INVALID (no blocks, hydro context, null entry in out), NOMEM,
 * DEVICE. */
amrvac_status amrvac_divb(amrvac_ctx *ctx, double *const *out, double *mean_abs_out);

/* Advances every block by nsteps steps of `scheme` (Sect. 2.3).  The
 * interiors of the u buffers are overwritten with U^{n+nsteps}; ghost layers
 * are not written.  dt_fixed: host pointer to a fixed step > 0, or NULL to
 * use dt = cfl / max_blocks sum_d (c_max,d / dx_d) evaluated on U^n at the
 * start of every step (the multi-D form of the Sect. 4.4 bound dt < dx /
 * c_w).  t_inout: host pointer; in: start time, out: end time.  Non-NULL
 * t_inout synchronises the stream and reports device errors; NULL does
 * neither.  Errors: INVALID (no blocks, nsteps < 0, scheme unknown, cfl not
 * > 0 and finite when dt_fixed is NULL, *dt_fixed not > 0 and finite),
 * NONPHYSICAL (only when synchronising), DEVICE, NOMEM. */
amrvac_status amrvac_ssprk_step(amrvac_ctx *ctx, int scheme, double cfl, const double *dt_fixed,
                                int nsteps, double *t_inout);

/* Size, in doubles, of the fixed per-device array that holds the stage
 * buffers of amrvac_ssprk_step_noalloc (64 MiB). */
#define AMRVAC_NOALLOC_MAX_DOUBLES 8388608

/* For callers that cannot allocate device memory while they step: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results (bit for bit) as amrvac_ssprk_step,
 * with two differences: its three stage buffers (A, B and the SSPRK(5,4)
 * accumulator S, each nvar x (total interior cells) doubles rounded up to a
 * multiple of 32) live in a fixed library-owned device array of
 * AMRVAC_NOALLOC_MAX_DOUBLES doubles instead of context scratch, and the
 * stages are launched one by one (no graph is built).  The call itself
 * allocates nothing (no hipMalloc, hipFree or allocating library routine);
 * every other buffer it uses was set up by amrvac_create and
 * amrvac_set_blocks.  The array exists once per device, is shared by every
 * context on that device and is held until the process ends; nothing in it
 * has to start at zero (every stage writes the buffer it hands on before a
 * later stage reads it).  Calls on one device whose streams overlap in time
 * race on the array: the caller must order them.
 * Errors: those of amrvac_ssprk_step; INVALID when the three stage buffers
 * need more than AMRVAC_NOALLOC_MAX_DOUBLES doubles (nothing enqueued,
 * state unchanged); DEVICE when the array's address could not be resolved
 * on this device at amrvac_create. */
amrvac_status amrvac_ssprk_step_noalloc(amrvac_ctx *ctx, int scheme, double cfl, const double *dt_fixed,
                                        int nsteps, double *t_inout);

/* Reverse mode of amrvac_ssprk_step at a fixed dt: with U_0 the current
 * block states (read only, not modified) and U_N the state after nsteps
 * steps, lam[b] (host array of nblocks device pointers, each in the padded
 * block layout) holds on entry dJ/dU_N (ghost entries ignored) and on
 * return dJ/dU_0 in the interiors; the face ghost layers of fixed faces
 * (nbr = -1) receive dJ/d(boundary data), the derivative with respect to
 * the caller's ghost values, which enter every stage of every step; every
 * other ghost entry (periodic faces, edges, corners) is set to 0.  The map
 * differentiated is the discrete scheme of Sects. 2.1-2.3 with c_max a
 * function of every stage state (its derivative is delivered to the
 * maximising cell, lowest block then lowest cell index on ties); MP5,
 * LIM03, minmod and median are differentiated along the branch taken by the
 * forward pass.  Checkpoints of U are kept every ckpt_every steps and the
 * steps in between are recomputed, segment by segment; on lists of at most
 * 2 x 256 tiles the next segment is recomputed on a second stream of the
 * context while the current one is reversed (twice the segment's stage
 * states and codes; environment variable AMRVAC_ADJOINT_OVERLAP=0/1 forces
 * it off or on; the result is the same bit for bit).  The context keeps the
 * state slots for later calls.  Requires n[d] >= 5 for every block and every
 * face neighbour.  Synchronises the stream and reports device errors.
 * Errors: INVALID (no blocks, null lam or entry, nsteps < 0, ckpt_every < 1,
 * dt not > 0 and finite, scheme unknown), UNSUPPORTED (n[d] < 5, GLM, Hall
 * MHD, passive blocks), NONPHYSICAL, NOMEM, DEVICE. */
amrvac_status amrvac_ssprk_adjoint(amrvac_ctx *ctx, int scheme, double dt, int nsteps,
                                   int ckpt_every, double *const *lam);

/* Dynamic grid activation (the paper's appendix "Dynamic grid
 * activation"), the host-side list building: a block is active when
 * want[b] != 0 (the caller's criterion); then, `safety` times, every passive
 * block with an active face neighbour becomes active (the safety belt; each
 * pass works on the flags the previous pass produced).  blocks: the block
 * list (only nbr is read); want, active_out: host arrays of nblocks bytes;
 * active_out receives 1 (active) or 0 (passive).  Returns the number of
 * active blocks, or -1 for invalid arguments (a null pointer, nblocks < 1,
 * safety < 0, a neighbour index outside [-1, nblocks)).  Makes no HIP call
 * and needs no device. */
int amrvac_activation_flags(const amrvac_block *blocks, int nblocks, const unsigned char *want,
                            int safety, unsigned char *active_out);

/* Dynamic grid activation, integration side: later amrvac_fd_rhs and
 * amrvac_ssprk_step calls evaluate and advance only the blocks with
 * active[b] != 0 (host array of nblocks bytes; NULL = every block, the
 * state after amrvac_set_blocks).  c_max and the time step are taken over
 * the active blocks' cells and cell widths.  Passive blocks are not
 * written: their current interiors are read at the start of every
 * amrvac_ssprk_step call and serve, unchanged through all stages, as halo
 * for active neighbours; amrvac_fd_rhs leaves their rhs arrays untouched.
 * Rebuilds the work list and drops cached graphs.  amrvac_autotune and
 * amrvac_ssprk_adjoint return UNSUPPORTED while a block is passive.
 * Errors: INVALID (no blocks, no active block), NOMEM, DEVICE. */
amrvac_status amrvac_set_active(amrvac_ctx *ctx, const unsigned char *active);

/* Waits for the context stream and returns (and clears) the sticky device
 * error: OK, NONPHYSICAL or DEVICE. */
amrvac_status amrvac_sync(amrvac_ctx *ctx);

/* Message describing the last error of ctx ("" if none); NULL ctx gives a
 * static description of context-less failures.  Owned by the library. */
const char *amrvac_last_error(const amrvac_ctx *ctx);

/* Releases the context and everything it owns (never the caller's
 * buffers).  NULL is ignored. */
void amrvac_destroy(amrvac_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* AMRVAC_H */
