/*
 * fdbb.h -- C ABI of the MI355X (gfx950) library for the compressible-Euler
 * building blocks of "FDBB: Fluid Dynamics Building Blocks" (Moeller,
 * Jaeschke).  Every entry point evaluates one building block point by point
 * over structure-of-arrays state vectors in a single pass over HBM.
 *
 * ---------------------------------------------------------------- notation
 * D = dim in {1, 2, 3} space dimensions, K = D + 2 state components.
 * Conservative state U = (rho, m_1..m_D, E): density, momentum rho v and
 * total energy per unit volume (the paper's "rho E"; Sec. 2.2, "Variables").
 * Primitive state V = (rho, v_1..v_D, p).  Perfect gas with adiabatic index
 * gamma = c_p / c_v > 1 (the paper's example: 7/2 over 5/2 = 1.4); only the
 * general EOS entry point (fdbb_eos_pvt) takes another equation of state.
 *
 * ---------------------------------------------------------------- layout
 * A "field set" is a device base pointer plus a leading dimension ld, in
 * elements: component k of point i is base[k * ld + i] (SoA), ld >= n.
 * The flux tensor is N_U x N_D row-major (Sec. 2.1, "Block Expressions":
 * row-major block storage; Sec. 2.2, "Inviscid Fluxes": the 5 x 3 block), so
 * flux component r of direction d is field r * D + d.  Flux Jacobian blocks
 * are point-major and row-major: entry (r, c) of A_d at point i is
 * A[(d * ldA + i) * K * K + r * K + c].
 *
 * dtype selects the storage type of every array of a call: FDBB_F64 (double)
 * or FDBB_F32 (float).  Arithmetic is FP64 in both cases; FP32 values are
 * widened exactly on load and rounded to nearest on store.
 *
 * ---------------------------------------------------------------- contract
 * Ownership: the caller owns every buffer; no entry point allocates or frees
 * memory, except the batch plans below, which own their descriptor tables
 * and graphs until destroyed (and the request server of fdbb_server.h,
 * which owns its arena).
 * Streams: `stream` is a hipStream_t passed as void*, NULL for the default
 * stream.  Calls are asynchronous: they validate on the host, enqueue one
 * kernel on `stream` and return; results are ready when the stream reaches
 * that point.  Only launch errors are reported, not asynchronous faults.
 * Validation (host side, before any HIP call):
 *   FDBB_EINVAL  dim not in {1,2,3}, gamma not finite or <= 1, unknown dtype,
 *                n < 0 or n >= 2^31 (FDBB_MAX_POINTS: a larger set is split
 *                into calls by the caller), a direction out of range, a NULL
 *                required pointer with n > 0, or ld < n;
 *   FDBB_EALIGN  a base pointer not aligned to its element size;
 *   FDBB_EALIAS  any overlap between an input and an output field set, or
 *                between two outputs, except the exact in-place use (same
 *                base, same ld) allowed for the K -> K transforms
 *                (cons2prim, prim2cons, cons2char, char2cons, char_apply,
 *                roe_average).  In place,
 *                cons2prim and prim2cons leave rho where it is and do not
 *                store it again (Sec. 2.2, "Variables": source and
 *                destination being the same costs no transfer of density);
 *   FDBB_EHIP    the HIP runtime reported an error at launch
 *                (fdbb_last_error() has its text).
 * n == 0 returns FDBB_OK without launching.  States that are not admissible
 * (rho <= 0, p < 0) are not errors: results follow IEEE arithmetic (NaN/Inf).
 * All entry points are thread-safe and re-entrant.
 */
#ifndef FDBB_H
#define FDBB_H

#include <stdint.h>

/* Points per call (and per batch task) are below this bound.  Offsets and
 * leading dimensions are 64-bit, so a call's arrays may span any size. */
#define FDBB_MAX_POINTS ((int64_t)1 << 31)

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { FDBB_F64 = 0, FDBB_F32 = 1 } fdbb_dtype;

typedef enum {
    FDBB_OK = 0,
    FDBB_EINVAL = 1,
    FDBB_EALIGN = 2,
    FDBB_EALIAS = 3,
    FDBB_EHIP = 4,
    FDBB_ENOMEM = 5
} fdbb_status;

/* Operation ids, used by fdbb_set_launch_config and the batch tasks. */
typedef enum {
    FDBB_OP_CONS2PRIM = 0,
    FDBB_OP_PRIM2CONS = 1,
    FDBB_OP_EOS = 2,
    FDBB_OP_FLUX = 3,
    FDBB_OP_FLUX_JACOBIAN = 4,
    FDBB_OP_RIEMANN = 5,
    FDBB_OP_CONS2CHAR = 6,
    FDBB_OP_CHAR2CONS = 7,
    FDBB_OP_FUSED = 8,
    FDBB_OP_ADJOINT = 9,
    FDBB_OP_V_MAG2 = 10,
    FDBB_OP_EIGENVECTORS = 11,
    FDBB_OP_CHAR_APPLY = 12,
    FDBB_OP_ROE_AVERAGE = 13,
    FDBB_OP_EOS_PVT = 14,
    FDBB_OP_VISCOUS_FLUX = 15,
    FDBB_OP_FLUX_DIR = 16,
    FDBB_NUM_OPS = 17
} fdbb_op;

/* Conservative -> primitive (Sec. 2.2, "Variables", conversion figure):
 * V = (rho, v = m / rho, p = (gamma-1)(E - rho |v|^2 / 2)).
 * U: K input fields; V: K output fields.  V == U (same ld) converts in place. */
int fdbb_cons2prim(int dim, double gamma, int dtype, const void *U, int64_t ldU,
                   void *V, int64_t ldV, int64_t n, void *stream);

/* Primitive -> conservative (Sec. 2.2, "Variables"):
 * U = (rho, rho v, p / (gamma-1) + rho |v|^2 / 2).  U == V converts in place. */
int fdbb_prim2cons(int dim, double gamma, int dtype, const void *V, int64_t ldV,
                   void *U, int64_t ldU, int64_t n, void *stream);

/* Squared velocity magnitude, the expression of the paper's micro-benchmark
 * (Sec. 3, Eq. 2): y[i] = (m . m) / (rho rho).  Reads rho and m (fields
 * 0..D of U; E is not touched) and writes one field of n elements. */
int fdbb_velocity_magnitude2(int dim, int dtype, const void *U, int64_t ldU, void *y, int64_t n,
                             void *stream);

/* Equation of state of the perfect gas (Sec. 2.2, "Equations of state";
 * the pressure is the p_rhoe member of the EOS prototype, p = (gamma-1) rho e):
 * p[i] and the speed of sound c[i] = sqrt(gamma p / rho), each a single
 * field of n elements.  Either output may be NULL (not both). */
int fdbb_eos(int dim, double gamma, int dtype, const void *U, int64_t ldU,
             void *p, void *c, int64_t n, void *stream);

/* Inviscid flux tensor (Sec. 2.2, "Inviscid Fluxes"):
 * F(U) = [rho v; rho v (x) v + I p; v (rho E + p)], K x D row-major:
 * F has K * D fields, field r * D + d = component r of F_d. */
int fdbb_flux(int dim, double gamma, int dtype, const void *U, int64_t ldU,
              void *F, int64_t ldF, int64_t n, void *stream);

/* The flux of one direction alone (Sec. 2.2, "Inviscid Fluxes": column `dir`
 * of the K x D flux block): F_dir = (m_dir, m v_dir + e_dir p, v_dir (E + p)).
 * Fd has K fields, field r = component r of F_dir; reads K fields and writes
 * K, where fdbb_flux writes K * D.  0 <= dir < dim, else FDBB_EINVAL. */
int fdbb_flux_direction(int dim, int dir, double gamma, int dtype, const void *U, int64_t ldU,
                        void *Fd, int64_t ldFd, int64_t n, void *stream);

/* Flux Jacobians A_d = dF_d / dU for d = 0..D-1 (Fig. 1, "flux-Jacobians";
 * the paper leaves them unfinished, Sec. 2.2, "Inviscid Fluxes"; these are
 * the exact analytic derivatives in conservative variables).  A holds D
 * point-major row-major K x K blocks per point, see the layout above;
 * ldA >= n is the per-direction block stride in points. */
int fdbb_flux_jacobian(int dim, double gamma, int dtype, const void *U, int64_t ldU,
                       void *A, int64_t ldA, int64_t n, void *stream);

/* Riemann invariants (Fig. 1): for each direction d the pair
 * w-_d = v_d - 2c/(gamma-1), w+_d = v_d + 2c/(gamma-1), then the entropy
 * s = p / rho^gamma.  R has 2D + 1 fields: (w-_0, w+_0, ..., w+_{D-1}, s). */
int fdbb_riemann_invariants(int dim, double gamma, int dtype, const void *U, int64_t ldU,
                            void *R, int64_t ldR, int64_t n, void *stream);

/* Characteristic variables of direction dir (Fig. 1; EnumForm
 * "characteristic", Sec. 2.2, "Variables"), taken pointwise as
 * W = (w-_dir, s, v_j for j != dir ascending, w+_dir): the invariants ordered
 * by the eigenvalues v_dir - c, v_dir (D times), v_dir + c of A_dir.
 * K fields in, K fields out; W == U converts in place. */
int fdbb_cons2char(int dim, int dir, double gamma, int dtype, const void *U, int64_t ldU,
                   void *W, int64_t ldW, int64_t n, void *stream);

/* Inverse of fdbb_cons2char: v_dir = (w+ + w-)/2, c = (gamma-1)(w+ - w-)/4,
 * rho = (c^2 / (gamma s))^(1/(gamma-1)), p = rho c^2 / gamma, then U. */
int fdbb_char2cons(int dim, int dir, double gamma, int dtype, const void *W, int64_t ldW,
                   void *U, int64_t ldU, int64_t n, void *stream);

/* Fused pass: the flux tensor (as fdbb_flux), the flux Jacobians (as
 * fdbb_flux_jacobian) and the Riemann invariants (as
 * fdbb_riemann_invariants) of the same state in one pass over U.  Any of
 * F, A, R may be NULL (not all). */
int fdbb_euler_fused(int dim, double gamma, int dtype, const void *U, int64_t ldU,
                     void *F, int64_t ldF, void *A, int64_t ldA, void *R, int64_t ldR,
                     int64_t n, void *stream);

/* Adjoint of the flux map: Ubar = sum_d A_d(U)^T Fbar_d (dir == -1; Fbar has
 * the flux tensor's K * D fields) or Ubar = A_dir(U)^T Fbar (dir in [0, D);
 * Fbar has K fields).  A_d is never formed.  Ubar has K fields. */
int fdbb_flux_adjoint(int dim, int dir, double gamma, int dtype, const void *U, int64_t ldU,
                      const void *Fbar, int64_t ldFbar, void *Ubar, int64_t ldUbar,
                      int64_t n, void *stream);

/* Linearised characteristic decomposition A_d = R_d diag(v_d - c, v_d (D
 * times), v_d + c) L_d of every direction (Fig. 1, "characteristic
 * variables", in the linearised form that characteristic boundary
 * conditions and limiters use).  The columns of R_d are the right
 * eigenvectors, in the order of the characteristic variables of
 * fdbb_cons2char: r- = (1, v - c e_d, H - c v_d), r0 = (1, v, |v|^2/2),
 * r_j = (0, e_j, v_j) for j != d ascending, r+ = (1, v + c e_d, H + c v_d),
 * with H = (E + p)/rho; L_d = R_d^{-1} in closed form.  Both are stored like
 * the Jacobian blocks (point-major, row-major K x K, per-direction stride
 * ldL / ldR points); either may be NULL (not both). */
int fdbb_eigenvectors(int dim, double gamma, int dtype, const void *U, int64_t ldU, void *L, int64_t ldL,
                      void *R, int64_t ldR, int64_t n, void *stream);

/* Y = L_dir(U) X (mode 0: increments of the state to characteristic
 * increments) or Y = R_dir(U) X (mode 1: back); X and Y have K fields.
 * Y == X (same ld) works in place.  Not available as a batch task. */
int fdbb_char_apply(int dim, int dir, int mode, double gamma, int dtype, const void *U, int64_t ldU,
                    const void *X, int64_t ldX, void *Y, int64_t ldY, int64_t n, void *stream);

/* Roe-averaged state between a left state UL and a right state UR, the
 * point at which the characteristic decomposition between two states is
 * linearised (Fig. 1, "characteristic variables"; Roe's average for the
 * perfect gas): with a = sqrt(rho_L), b = sqrt(rho_R), rho^ = a b, v^ and
 * H^ = (E + p)/rho averaged with weights a and b, written as the conservative
 * state Uh = (rho^, rho^ v^, rho^ H^ - p^), p^ = (gamma-1)/gamma rho^ (H^ -
 * |v^|^2/2).  The Jacobians at Uh satisfy A_d(Uh)(UR - UL) = F_d(UR) -
 * F_d(UL); fdbb_eigenvectors and fdbb_char_apply take Uh as their state.
 * UL, UR and Uh have K fields each; Uh may be UL or UR (same base and ld:
 * in place).  Also a batch task (in0 = UL, in1 = UR, out0 = Uh). */
int fdbb_roe_average(int dim, double gamma, int dtype, const void *UL, int64_t ldUL, const void *UR,
                     int64_t ldUR, void *Uh, int64_t ldUh, int64_t n, void *stream);

/* Equations of state of the form f(p, V, T) = 0 behind a runtime id (Sec.
 * 2.2, "Equations of state": each supplies p(rho, e) and T(rho, e), e the
 * specific internal energy e = E/rho - |v|^2/2).  Per point: pressure p,
 * speed of sound c (the isentropic derivative of p) and temperature T.
 *   eos FDBB_EOS_PERFECT_GAS, params = {c_p, c_v} (c_p > c_v > 0):
 *     gamma = c_p/c_v, p = (gamma-1) rho e, T = e/c_v, c^2 = gamma p/rho;
 *   eos FDBB_EOS_STIFFENED_GAS, params = {gamma, p_inf, c_v} (gamma > 1,
 *     p_inf >= 0, c_v > 0): p = (gamma-1) rho e - gamma p_inf,
 *     T = (e - p_inf/rho)/c_v, c^2 = gamma (p + p_inf)/rho.
 * p, c, T are single fields of n values, any of them NULL (not all).  Not a
 * batch task (tasks carry gamma only). */
typedef enum { FDBB_EOS_PERFECT_GAS = 0, FDBB_EOS_STIFFENED_GAS = 1 } fdbb_eos_id;
int fdbb_eos_pvt(int dim, int eos, const double *params, int dtype, const void *U, int64_t ldU, void *p,
                 void *c, void *T, int64_t n, void *stream);

/* Viscous flux tensor (Fig. 1, "viscous fluxes", named there without a
 * definition; this is the compressible Navier-Stokes one): Newtonian stress
 * with Stokes' hypothesis and Fourier heat conduction, constant dynamic
 * viscosity mu >= 0 and conductivity kappa >= 0:
 *   tau_ij = mu (dv_i/dx_j + dv_j/dx_i) - (2/3) mu delta_ij div v,
 *   F^v_d  = (0, tau_1d .. tau_Dd, sum_j v_j tau_jd + kappa dT/dx_d).
 * Inputs: U (K fields; v = m/rho), the velocity gradient G (D*D fields,
 * field i*D + j = dv_i/dx_j) and the temperature gradient gradT (D fields).
 * Fv has the flux tensor's K*D fields (field r*D + d; the mass row is
 * written as zeros).  Not a batch task. */
int fdbb_viscous_flux(int dim, double mu, double kappa, int dtype, const void *U, int64_t ldU, const void *G,
                      int64_t ldG, const void *gradT, int64_t ldGT, void *Fv, int64_t ldFv, int64_t n,
                      void *stream);

/* ---------------------------------------------------------------- tuning
 * Launch configuration per (op, dim, dtype): `block` threads per workgroup
 * (64..1024, a multiple of 64; at most 256 for the flux Jacobian and the
 * fused pass, whose kernels stage blocks in LDS), `ppt` points per thread
 * (1, 2 or 4), `grid_cap` the largest grid (0 = one tile per workgroup;
 * otherwise workgroups loop over tiles) and `nontemporal` (1: outputs are
 * written with streaming stores, 0: regular stores; a streaming store sets
 * the nt cache-policy bit, and in the fused pass, flux Jacobian,
 * eigenvector blocks, flux and Riemann invariants, in FP64 cons2prim and
 * prim2cons and in FP32 |v|^2 also sc1, the device-scope bit).  Returns
 * FDBB_EINVAL for values outside these sets.  The table is process-wide and
 * safe to update while other threads launch. */
int fdbb_set_launch_config(int op, int dim, int dtype, int block, int ppt, int grid_cap,
                           int nontemporal);
int fdbb_get_launch_config(int op, int dim, int dtype, int *block, int *ppt, int *grid_cap,
                           int *nontemporal);

/* A second configuration per (op, dim, dtype) for small launches: a call of
 * n <= max_n points uses it instead of the one above (a grid of few tiles
 * pays its ramp-up and tail on every launch, so a different shape can win
 * there).  The values are validated as above; max_n = 0 removes the entry
 * (the other arguments are then not checked) and a negative max_n gives
 * FDBB_EINVAL.  Process-wide, safe to update while other threads launch: a
 * launch racing an update takes either the old or the new entry. */
int fdbb_set_small_launch_config(int op, int dim, int dtype, int64_t max_n, int block, int ppt,
                                 int grid_cap, int nontemporal);
/* max_n 0 and the large configuration's values when no entry is set. */
int fdbb_get_small_launch_config(int op, int dim, int dtype, int64_t *max_n, int *block, int *ppt,
                                 int *grid_cap, int *nontemporal);
/* The configuration a call of n points of (op, dim, dtype) launches with
 * (outputs may be NULL); n < 0 gives FDBB_EINVAL. */
int fdbb_launch_config_for(int op, int dim, int dtype, int64_t n, int *block, int *ppt, int *grid_cap,
                           int *nontemporal);

/* Resources of the kernel that (op, dim, dtype, ppt, nontemporal) launches:
 * vector registers per thread and private (spill) bytes per thread, which
 * cost memory traffic when non-zero.  Either output may be NULL.  Queries
 * the HIP runtime (FDBB_EHIP if that fails). */
int fdbb_kernel_info(int op, int dim, int dtype, int ppt, int nontemporal, int *vgprs,
                     int *scratch_bytes);

/* ---------------------------------------------------------------- batches
 * Many independent blocks of uneven size in one persistent launch.  A task
 * names one operation on one field-set group; its fields mean what the
 * matching single-call entry point's arguments mean:
 *   in0  = U (V for prim2cons, W for char2cons), in1 = Fbar (adjoint only),
 *   out0 = V / U / p / F / F_dir / A / R / W / Ubar / y (v_mag2), out1 = c (eos) or A (fused),
 *   out2 = R (fused).  Unused pointers are NULL. */
typedef struct {
    int32_t op;     /* fdbb_op */
    int32_t dim;
    int32_t dtype;  /* fdbb_dtype */
    int32_t dir;    /* direction for cons2char/char2cons/adjoint/flux_dir, else 0 */
    double gamma;
    int64_t n;
    const void *in0;
    int64_t ld_in0;
    const void *in1;
    int64_t ld_in1;
    void *out0;
    int64_t ld_out0;
    void *out1;
    int64_t ld_out1;
    void *out2;
    int64_t ld_out2;
} fdbb_task;

/* Validate one task as its single-call entry point would (no HIP call).
 * FDBB_EINVAL for FDBB_OP_EOS_PVT and FDBB_OP_VISCOUS_FLUX, whose
 * parameters and inputs a task cannot carry. */
int fdbb_task_check(const fdbb_task *task);

/* Run one task through its single-call entry point on `stream` (char_apply
 * tasks apply L; FDBB_OP_EOS_PVT and FDBB_OP_VISCOUS_FLUX are refused as
 * above). */
int fdbb_task_run(const fdbb_task *task, void *stream);

typedef struct fdbb_batch_plan fdbb_batch_plan;

/* Create a plan for up to `capacity` tasks (>= ntasks) and load `tasks`
 * into it.  Each task is validated as its single-call entry point would be.
 * The plan owns a device copy of the task table, the tile prefix sums and a
 * HIP graph holding one persistent kernel with `grid` workgroups of `block`
 * threads (64..256 in multiples of 64; grid 0 picks one sized to the
 * device), `ppt` points per thread (1, 2, 4 or 8) and regular (0),
 * streaming (1: the nt bit) or streaming device-coherent (2: nt and sc1)
 * output stores.  block == 0 takes the batch configuration installed for
 * the first task's storage type (FDBB_F64 for an empty list; see
 * fdbb_set_batch_config) and ignores ppt, grid and nontemporal.  Tasks that
 * overlap one another's outputs are rejected (FDBB_EALIAS).  Jacobian
 * staging needs LDS; a plan holds what its first task list needs, or, when
 * created with ntasks == 0, what any task needs (later task lists needing
 * more than the plan holds are rejected with FDBB_EINVAL).  Every op but
 * FDBB_OP_EIGENVECTORS, FDBB_OP_CHAR_APPLY, FDBB_OP_EOS_PVT and
 * FDBB_OP_VISCOUS_FLUX can be a task (FDBB_EINVAL otherwise). */
int fdbb_batch_plan_create(const fdbb_task *tasks, int ntasks, int capacity, int block,
                           int ppt, int grid, int nontemporal, fdbb_batch_plan **plan);

/* Replace the task list (ntasks <= capacity); stream-ordered on `stream`:
 * the upload happens before any later fdbb_batch_exec on the same stream. */
int fdbb_batch_plan_update(fdbb_batch_plan *plan, const fdbb_task *tasks, int ntasks,
                           void *stream);

/* Run the plan's persistent launch on `stream`: use_graph != 0 replays the
 * captured HIP graph, 0 launches the same kernel directly.  The graph was
 * captured with the LDS the plan reserved at creation (a plan created empty
 * reserves 3D FP64 Jacobian staging, which leaves room for one or two
 * workgroups per compute unit); a direct launch takes only what the current
 * task list stages, none for a list without Jacobian blocks. */
int fdbb_batch_exec(fdbb_batch_plan *plan, void *stream, int use_graph);

/* The batch configuration that plans created with block == 0, the
 * allocation-free batch entry point with block == 0 and the request server
 * use, per storage type: block (64..256, multiple of 64), ppt (1, 2, 4, 8),
 * grid_per_cu workgroups per compute unit (0: 2048 / block; at most 1024),
 * store mode nontemporal (0, 1, 2 as for plans).  The binding installs the autotuned
 * table's entry at load; until then 256 threads, 1 point per thread, the
 * default grid and streaming stores.  FDBB_EINVAL for values out of range
 * or a configuration whose 3D Jacobian staging would not fit in LDS. */
int fdbb_set_batch_config(int dtype, int block, int ppt, int grid_per_cu, int nontemporal);
int fdbb_get_batch_config(int dtype, int *block, int *ppt, int *grid_per_cu, int *nontemporal);

/* The batch configuration of the request server's batched launches, whose
 * task mix (small requests of every op, dim and storage type) wants another
 * shape than a batch of fused passes.  Same ranges and checks as
 * fdbb_set_batch_config (3D FP64 Jacobian staging must fit); block 0
 * removes the entry, and until one is installed the server takes the FP64
 * batch configuration, which the getter then reports.  Servers read it when
 * they are created. */
int fdbb_set_server_batch_config(int block, int ppt, int grid_per_cu, int nontemporal);
int fdbb_get_server_batch_config(int *block, int *ppt, int *grid_per_cu, int *nontemporal);

/* The launch configuration a plan was created with (any may be NULL). */
int fdbb_batch_plan_config(const fdbb_batch_plan *plan, int *block, int *ppt, int *grid,
                           int *nontemporal);

/* Total points and tiles of the current task list (either may be NULL). */
int fdbb_batch_plan_info(const fdbb_batch_plan *plan, int64_t *points, int64_t *tiles);

/* Free the plan (waits for nothing: the caller must make sure no launch of
 * it is still running). */
int fdbb_batch_plan_destroy(fdbb_batch_plan *plan);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): one persistent batch launch of `tasks`
 * with the meaning of fdbb_batch_plan_create + fdbb_batch_exec(use_graph =
 * 0), without a plan.  Allocates nothing: the task table goes into a fixed
 * device array of the library, one per device (about 230 KB, held until the
 * process ends), with room for FDBB_NOALLOC_MAX_TASKS tasks; more tasks give
 * FDBB_EINVAL.  Tasks, block (64..256, or 0 for the installed batch
 * configuration), ppt, grid (0 picks one sized to the device) and
 * nontemporal are validated as for a plan, with the same statuses; each
 * call uploads only its own table, nothing needs clearing.
 * The table is copied from the library's static host staging array, a copy
 * that HIP completes before returning (pageable host memory), so the call
 * waits for the work already queued on `stream`; it is therefore not for
 * use under stream capture.  The kernel reads the table when it runs: calls
 * on one stream are ordered, but calls on one device that overlap in time
 * from different streams race on the shared table. */
#define FDBB_NOALLOC_MAX_TASKS 1024
int fdbb_batch_run_noalloc(const fdbb_task *tasks, int ntasks, int block, int ppt, int grid,
                           int nontemporal, void *stream);

/* ---------------------------------------------------------------- misc */
const char *fdbb_status_string(int status);
/* Text of the last error reported on the calling thread ("" if none). */
const char *fdbb_last_error(void);
/* Library version, major * 10000 + minor * 100 + patch. */
int fdbb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FDBB_H */
