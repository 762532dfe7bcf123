/*
 * mbstokes.h - C ABI of the many-body active-sphere Stokes solver (MI355X / gfx950).
 *
 * Method: Galerkin discretisation of the boundary-integral equation of Stokes
 * flow for N spheres of radius a with active (Dirichlet) slip, Singh, Ghose &
 * Adhikari, "Many-body microhydrodynamics of colloidal particles with active
 * boundary layers" (arXiv:1411.0278).
 *
 *   - Known lower traction coefficients: the contact force and torque balance
 *     the body force F^e and torque T^e (section II, overdamped Newton's
 *     equations as constraints).
 *   - Unknown higher coefficients kept at this truncation (traction ranks <= 2,
 *     i.e. force, torque and stresslet): the flow stresslet
 *     Sigma_n = a Q^(20)_n (section IV, named combinations), 5 per sphere.
 *   - Linear system: the symmetric l = 1 Galerkin rows (section II, Schur
 *     "higher" rows; section III, off-diagonal matrix elements as derivatives of
 *     the Green's function with the finite-size operators F^l):
 *        Sigma_n / gamma - sum_{m != n} E[Sigma_m] = sum_{m != n} E[F, T, d] - c s_n,
 *     gamma = (20/3) pi eta a^3, solved matrix-free by GMRES.
 *   - Outputs: rigid-body motion by the generalized Stokes laws (section III),
 *        V_n = V^a_n + F^e_n/(6 pi eta a) + sum_{m != n} U[F, T, Sigma, d],
 *        Omega_n = T^e_n/(8 pi eta a^3) + sum_{m != n} W[F, T, Sigma],
 *     with V^a_n = -V^(1s)_n, and the traction stresslet S_n = Sigma_n + (8/3) pi eta a^3 s_n.
 *   - The _ex entry points add the septlet, vortlet and spinlet slip modes of the
 *     minimal truncation (section IV) as further fixed sources in E, U and W.
 *   - The _r3 entry points solve the traction rank <= 3 system of the minimal
 *     truncation instead: the septlet, vortlet and potential-dipole traction modes
 *     are unknowns beside the stresslet, with the quadratic (l = 2) surface
 *     conditions as their rows (20 unknowns per sphere; declared below).
 *
 * Conventions for every entry point below:
 *   - Arrays are caller-owned, contiguous, row-major, particle-major, IEEE
 *     binary64, and live in DEVICE memory of the context's GPU (for example
 *     torch.float64 CUDA tensors). Vectors are [n x 3]; symmetric traceless
 *     rank-2 quantities (s, Sigma, S, strains) are [n x 5] in the orthonormal
 *     basis  B0 = (xx - yy)/sqrt2, B1 = (2zz - xx - yy)/sqrt6,
 *     B2 = (xy + yx)/sqrt2, B3 = (xz + zx)/sqrt2, B4 = (yz + zy)/sqrt2.
 *   - Optional inputs may be NULL, meaning zero.
 *   - Work is enqueued on `stream` (NULL = the default stream); every call
 *     returns after its work on that stream has completed.
 *   - An output array must not share memory with an input or with another output
 *     (MBS_EINVAL, checked on the address ranges before any work).
 *   - Orientations p, wherever an entry point reads them, must be unit vectors:
 *     | |p| - 1 | <= 1e-12 for every row (MBS_EINVAL otherwise).
 *   - Return value: MBS_OK or a negative error code; the message for the last
 *     failure on the context is available from mbs_last_error. No C++
 *     exception crosses this interface. On an error no output is written
 *     unless the description says otherwise.
 *   - A context may be used by one host thread at a time; calls on one context
 *     are serialised by the caller.
 */
#ifndef MBSTOKES_H
#define MBSTOKES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MBS_OK            0
#define MBS_EINVAL       -1  /* bad argument: NULL required pointer, n < 1, bad option, non-finite value,
                                orientation p with | |p| - 1 | > 1e-12, output overlapping an input */
#define MBS_ENOCONV      -2  /* iteration cap reached; outputs hold the last iterate, stats->rel_resid is set */
#define MBS_EOVERLAP     -3  /* two centres closer than 2a (only when check_overlap is set) */
#define MBS_EUNSUPPORTED -4  /* option not supported (for example lmax != 2) */
#define MBS_ENOMEM       -5  /* device allocation failed */
#define MBS_EHIP         -6  /* HIP runtime error; the HIP message is in mbs_last_error */

#define MBS_FP64   0   /* pair blocks and Krylov arithmetic in binary64 */
#define MBS_MIXED  1   /* binary32 pair blocks inside a binary64 iterative refinement; residuals
                          and corrections in binary64. Accumulation of the binary32 operator: plain
                          binary32 fused multiply-adds within a segment of sources (64 records, or
                          one LDS tile of 64-256), Kahan-compensated binary32 sums of the segment
                          totals, and binary64 sums of the source chunks */
#define MBS_FP32   1   /* precision selector of mbs_matvec: binary32 pair blocks */

#define MBS_GUESS_ZERO     0   /* Sigma^0 = 0 */
#define MBS_GUESS_DIAG     1   /* Sigma^0 = gamma b: the one-body (diagonal) solve of the system */
#define MBS_GUESS_LEARNED  2   /* Sigma^0 = gamma b + net(neighbourhood features); needs a network
                                  (mbs_warmstart_init/set/load/train), p and n >= 17
                                  (mbs_solve_batched always starts from zero) */
#define MBS_GUESS_USER     3   /* Sigma^0 = the caller's sigma0 */

typedef struct mbs_params {
  double  eta;           /* viscosity (> 0) */
  double  a;             /* sphere radius (> 0) */
  double  tol;           /* stop when ||b - A Sigma||_2 / ||b||_2 <= tol (binary64 residual) */
  double  self_slip_c;   /* c in "- c s_n": 1 = lone sphere meets its strain slip exactly;
                            1.4 reproduces the paper's one-body stresslet table */
  double  inner_tol;     /* MBS_MIXED: relative tolerance of each inner binary32 GMRES solve (an
                            inner solve also stops once its residual is below 0.3 tol |b|) */
  double  near_cutoff;   /* > 0: right-precondition GMRES with M^{-1} = gamma (I + X + ... + X^k), X =
                            gamma K_near (Neumann series of (I/gamma - K_near)^{-1} to the even
                            order k = near_order),
                            K_near the operator's blocks of pairs closer than near_cutoff (centre distance;
                            at most 32 neighbours per sphere, the smallest indices; pairs closer
                            than 2a are left out); 0 = no preconditioner (default). The solution
                            is unchanged. Applies to mbs_solve, mbs_step and mbs_solve_batched
                            (there within each configuration). */
  int32_t lmax;          /* traction truncation rank of these entry points: only 2 (force, torque,
                            stresslet); rank 3 has its own entry points (mbs_solve_r3) */
  int32_t max_iter;      /* cap on GMRES iterations (all restarts, inner iterations included) */
  int32_t restart;       /* GMRES restart length m, 1..64 */
  int32_t precision;     /* MBS_FP64 or MBS_MIXED */
  int32_t guess;         /* MBS_GUESS_* */
  int32_t check_overlap; /* nonzero: mbs_solve fails with MBS_EOVERLAP if some |R_n - R_m| < 2a
                            (two distinct spheres at one centre included);
                            zero: overlapping spheres are solved as given (the pair blocks hold for
                            any r > 0); two distinct spheres at one centre (r = 0) have infinite
                            pair blocks, so the pair passes return non-finite values for them and
                            mbs_solve ends with MBS_ENOCONV and a non-finite rel_resid */
  int32_t tile;          /* pair-kernel launch shape: 0 = autotuned (or default), k > 0 = entry k-1
                            of the candidate table (see mbs_autotune) */
  int32_t graph;         /* 1 (default): mbs_solve_batched captures its phases in HIP graphs and
                            replays them; mbs_solve / mbs_step with n <= 32768 capture the GMRES
                            Arnoldi steps from the second solve with the same sizes, positions
                            pointer and workspace on (operator timings t_op*_ms then cover only the
                            eagerly launched applications); 0 = launch the same kernels directly */
  int32_t batch_item;    /* mbs_solve_batched: receivers per work item (64, 128 or 256); 0 = the
                            context's choice (mbs_autotune_batched, else 64) */
  int32_t superposition; /* nonzero: mbs_solve and mbs_step use the superposition approximation of
                            section IV instead of solving: Sigma_n = -c gamma s_n (lone-sphere
                            stresslets), outputs by the direct sum; 0 = the many-body solve */
  int32_t near_order;    /* order k of the near-field preconditioner's Neumann series: 2 (default;
                            0 means 2), 4, 6 or 8 (even orders keep M^{-1} positive definite for
                            any near block); each order is one sparse pass over the neighbour lists */
  int32_t spatial_order; /* mbs_solve(_ex) and mbs_step work internally with the spheres in the Morton
                            order of their centres (inputs gathered into that order, outputs
                            scattered back, so the caller sees its own order): 0 = when n >= 65536
                            (default), 1 = always, -1 = never. A workgroup's receivers are then
                            neighbours in space, so binary32 coordinates relative to the first of
                            them stay small (N = 10^6: binary32 operator error 8.6e-7 -> 1.1e-7, one
                            binary32 iteration fewer); otherwise only the order of the sums, and so
                            the rounding, changes */
  int32_t plane;         /* 1: the fluid fills the half space z > plane_z above a flat plane on which it
                            slips freely (zero normal velocity and tangential stress: a flat free
                            surface). Its Green's function is the free-space one plus its mirror
                            image, so every sphere also acts through its mirror image in the plane
                            (on every sphere, itself included), with F* = M F, T* = -M T,
                            Sigma* = M Sigma M, d* = M d, M = diag(1, 1, -1). The images' part of the
                            operator runs in the pass's precision (binary32 in the inner passes of
                            MBS_MIXED); the right-hand side, outputs and flow add theirs in binary64.
                            2: the plane is a no-slip wall (zero velocity on it). Its Green's
                            function is Blake's: the free-space one plus an image system at the
                            mirror point (a Stokeslet, a Stokes doublet and a source doublet whose
                            strengths depend on the source's height); every sphere acts through it
                            on every sphere, itself included, with each source's finite-size operator
                            taken in the source point. Its image part runs in binary64 in every pass.
                            Both follow the paper's remark that other geometries, plane walls among
                            them, follow from their Green's function (Discussion). Every sphere must
                            lie at least a above the plane (MBS_EINVAL otherwise). Applies to
                            mbs_solve(_ex), mbs_matvec, mbs_rhs(_ex), mbs_outputs(_ex), mbs_flow(_ex)
                            (field points must lie in the fluid too) and mbs_step (which monitors
                            the heights, see there); the higher slip modes, the batched solver, the
                            rank <= 3 entry points and mbs_matvec_static refuse it
                            (MBS_EUNSUPPORTED). The near-field
                            preconditioner keeps the free-space pairs. 0 = unbounded fluid (default);
                            other values are MBS_EINVAL */
  int32_t ewald_mesh;    /* box > 0: 0 = the Fourier part of the Ewald sums directly over the wave
                            vectors (O(N K), the default); -1: M chosen as the smallest power of 2
                            from 16 to 512 with box/M <= 1.25 a; M = a power of 2 from 16 to 512: smooth
                            particle-mesh Ewald on an M^3 mesh of spacing box/M, the fast
                            matrix-vector product that the paper leaves to future work (section IV): every
                            sphere's coefficients spread onto the mesh by cardinal B-splines of
                            order 8, one 3D FFT, the same Fourier multipliers per mesh wave vector
                            (|m| < M/2 per axis), the inverse FFT interpolated back with the same
                            weights, so a pass costs O(N + M^3 log M) with the real-space part kept
                            within rc = 5/xi; ewald_xi defaults to pi M/(14 box), kept at most
                            0.5/a and at least 10/box, and an explicit xi * box must be at least 10.
                            The result carries the mesh's interpolation error, about 1e-6 of the
                            Fourier part at the default xi (smaller xi or larger M: smaller), instead
                            of the direct sums' 1e-13; it grows roughly as (xi a)^7 once xi a exceeds
                            about 0.5 (boxes under 20a). Device memory: 160 M^3
                            bytes of mesh fields plus about 270 bytes per sphere (and about 60 per
                            field point in mbs_flow). Other values are
                            MBS_EINVAL, as is a mesh without a box */
  double  plane_z;       /* height of the plane (plane != 0) */
  double  box;           /* > 0: the spheres fill a periodic cubic box of this side (the paper's remark
                            that periodic domains follow from the periodic Green's function, whose
                            direct sum converges only conditionally, Discussion). Hasimoto's
                            procedure: the fluid's mean velocity over the box is zero (the k = 0
                            Fourier mode is left out; a net force on the spheres is balanced by a
                            mean pressure gradient), and the periodic Oseen tensor is summed by
                            Ewald's method: a screened real-space part over the minimum image within
                            rc = 6.5/xi <= box/2 and a Fourier part over the reciprocal lattice up to
                            |k| = 13 xi, each sphere's own images through the Fourier sum less its
                            smooth self part; binary64 in every pass (truncation below 1e-13 of the
                            blocks). Positions may lie anywhere (they are taken modulo the box).
                            Applies to mbs_solve(_ex), mbs_matvec, mbs_rhs(_ex), mbs_outputs(_ex),
                            mbs_flow(_ex) without higher slip modes, and mbs_step (which leaves the
                            positions unwrapped and reports minimum-image distances in min_dist);
                            the batched solver, the rank <= 3 entry points, the warm-start calls and
                            mbs_matvec_static refuse it (MBS_EUNSUPPORTED); exclusive with plane
                            (MBS_EINVAL). The near-field preconditioner keeps its unwrapped
                            neighbour lists. 0 = unbounded fluid (default) */
  double  ewald_xi;      /* Ewald splitting parameter xi (box > 0): 0 = max(13, 13 (n/10^4)^0.15)/box
                            (balances the real-space pairs, which fall as (xi box)^-3, against the
                            wave vectors, which grow as (xi box)^3); larger values move work to the
                            Fourier sum; xi * box < 13 is MBS_EINVAL (the real-space cutoff 6.5/xi
                            must stay within box/2) */
} mbs_params;

typedef struct mbs_stats {
  int32_t iters;          /* GMRES iterations (Arnoldi steps), all restarts and refinements */
  int32_t refinements;    /* MBS_MIXED outer refinement steps */
  int32_t fp64_matvecs;   /* binary64 operator applications */
  int32_t fp32_matvecs;   /* binary32 operator applications */
  double  rel_resid;      /* final ||b - A Sigma||_2 / ||b||_2, evaluated in binary64 */
  double  t_total_ms;     /* device time of the whole call */
  double  t_rhs_ms;       /* right-hand side pass */
  double  t_iter_ms;      /* guess + iterations + refinement residuals (with the fused pass) */
  double  t_out_ms;       /* the pass that produced the rigid-body outputs */
  double  pair_blocks;    /* pair-block evaluations performed (all passes) */
  double  t_op64_ms;      /* summed device time of the binary64 operator applications */
  double  t_op32_ms;      /* summed device time of the binary32 operator applications */
  int32_t out_fused;      /* 1: the final binary64 residual and the outputs came from one fused pass
                             over the pairs (not counted in fp64_matvecs / t_op64_ms); 0: separate
                             output pass */
  int32_t reserved;
} mbs_stats;

typedef struct mbs_ctx mbs_ctx;

/* Fill *prm with the defaults: eta = 1/(6 pi), a = 1, tol = 1e-10, c = 1, inner_tol = 1e-5,
   lmax = 2, max_iter = 300, restart = 30, MBS_FP64, MBS_GUESS_ZERO, no overlap check, tile 0,
   graph 1, near_order 2, spatial_order 0, no plane, no box. */
void mbs_default_params(mbs_params* prm);

/* Create a context on HIP device `device`. *ctx receives the handle (NULL on failure).
   The context owns its device workspace (grown on demand, freed by mbs_destroy). */
int mbs_create(mbs_ctx** ctx, int device, const mbs_params* prm);
void mbs_destroy(mbs_ctx* ctx);
/* Replace the parameters of an existing context (validated as in mbs_create). */
int mbs_set_params(mbs_ctx* ctx, const mbs_params* prm);
/* Message of the last failure on ctx ("" if none); valid until the next call on ctx.
   With ctx == NULL: the message of the last failed mbs_create on this thread. */
const char* mbs_last_error(const mbs_ctx* ctx);

/* Full solve (sections II-III): Sigma from the stresslet rows, then V, Omega, S.
     R      [n x 3]  sphere centres
     p      [n x 3]  unit orientations (read by the learned warm start; may be NULL otherwise;
                     checked for unit length whenever given)
     v1s    [n x 3]  mean slip mode V^(1s); V^a = -V^(1s)
     v2s    [n x 5]  symmetric traceless linear slip mode s = V^(2s)
     v3t    [n x 3]  rank-3 trace slip mode d = V^(3t) (a fixed source, exterior flow
                     (a^5/10)(3 x^ x^ - I).d / r^3)
     Fe, Te [n x 3]  body force and torque
     sigma0 [n x 5]  initial guess for MBS_GUESS_USER (else ignored)
   Outputs: V, W (= Omega) [n x 3], S [n x 5] traction stresslet, Sigma [n x 5] flow stresslet
   (Sigma may be NULL). st may be NULL. MBS_ENOCONV still writes the outputs of the last iterate. */
int mbs_solve(mbs_ctx* ctx, int64_t n, const double* R, const double* p, const double* v1s,
              const double* v2s, const double* v3t, const double* Fe, const double* Te,
              const double* sigma0, double* V, double* W, double* S, double* Sigma,
              mbs_stats* st, void* stream);

/* The system operator (the GMRES matvec):  y_n = x_n / gamma - sum_{m != n} E[x_m](R_n - R_m),
   x, y [n x 5]: the stresslet rows of the Galerkin system, i.e. the off-diagonal matrix elements
   between the symmetric l = 1 modes of two spheres (section III, matrix elements as derivatives of
   the Green's function under the finite-size operators F^1 of both spheres) and the one-body
   diagonal 1/gamma (section IV, one-body traction-velocity relations, stresslet).
   precision: MBS_FP64 or MBS_FP32 (binary32 pair blocks, accumulated as described at MBS_MIXED;
   x and y stay binary64). y must not overlap x or R. The spheres are taken in the
   order given (no spatial reordering, see params.spatial_order): binary32 coordinates are rounded
   relative to the first receiver of each block of 256, so the binary32 error is smallest when
   neighbouring indices are neighbours in space. */
int mbs_matvec(mbs_ctx* ctx, int64_t n, const double* R, const double* x, double* y,
               int precision, void* stream);

/* mbs_matvec for callers that cannot allocate device memory (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): the same operator, launch shape and results as
   mbs_matvec, with every intermediate (chunk partial sums, packed source records, box centre) in a
   static 56 MiB device array of the library instead of the context's workspace. It calls no
   allocating routine. Limits: n <= 131072 (MBS_EINVAL beyond, or if the context's launch shape
   needs more scratch than the array holds; both checked before any work). Each GPU holds one copy
   of the array for the life of the process and every call on that GPU shares it, from any context:
   calls that overlap in time on one GPU (other streams, other host threads) race and give wrong
   results. Nothing from one call is read by the next. */
int mbs_matvec_static(mbs_ctx* ctx, int64_t n, const double* R, const double* x, double* y,
                      int precision, void* stream);

/* The near-field preconditioner on its own: y = gamma sum_{i <= k} (gamma K_near)^i x, k =
   params.near_order (x, y [n x 5] binary64 DEVICE, params.near_cutoff > 0; y must not overlap x or
   R). K_near holds the blocks of mbs_matvec's sum (section III off-diagonal stresslet elements)
   for the pairs on the neighbour lists; the series is the Neumann expansion of the inverse of the
   near part of the system, an addition of this library (the paper names no solver). */
int mbs_precond_apply(mbs_ctx* ctx, int64_t n, const double* R, const double* x, double* y, void* stream);

/* Right-hand side of the stresslet rows: b_n = sum_{m != n} E[F_m, T_m, d_m] - c s_n, b [n x 5]:
   the known lower coefficients (force and torque, section II, overdamped Newton's equations as
   constraints) and the fixed rank-3 trace mode moved to the right of the Schur "higher" rows
   (section II, lower/higher partition), with the elements of section III (strain of the
   Stokeslet with its finite-size operator F^0, of the rotlet and of the potential dipole) and the
   self slip term of section IV. b must not overlap any input. */
int mbs_rhs(mbs_ctx* ctx, int64_t n, const double* R, const double* v2s, const double* v3t,
            const double* Fe, const double* Te, double* b, void* stream);

/* Rigid-body outputs for a given flow stresslet Sigma [n x 5] (generalized Stokes laws):
   V, W [n x 3], S [n x 5] (S may be NULL). With Sigma = -c gamma s this is the paper's
   superposition approximation (section IV). */
int mbs_outputs(mbs_ctx* ctx, int64_t n, const double* R, const double* v1s, const double* v2s,
                const double* v3t, const double* Fe, const double* Te, const double* Sigma,
                double* V, double* W, double* S, void* stream);

/* Flow of the suspension at m field points X [m x 3] (section III: the exterior flow is the sum
   over spheres of the flows of their force F^e (with the finite-size factor 1 + a^2/6 nabla^2),
   torque (rotlet), flow stresslet Sigma (with 1 + a^2/10 nabla^2) and rank-3 trace mode d =
   V^(3t); no finite-size operator acts at the field point). Typically Sigma is the solution of
   mbs_solve for the same spheres. n, R, Fe, Te, Sigma, v3t: as in mbs_solve (Fe, Te, v3t may be
   NULL = zero). U: [m x 3]. Field points should lie outside every sphere (inside, the result is
   the exterior formula, not the rigid-body motion); a field point exactly on a centre gets no
   contribution from that sphere. */
int mbs_flow(mbs_ctx* ctx, int64_t m, const double* X, int64_t n, const double* R, const double* Fe,
             const double* Te, const double* Sigma, const double* v3t, double* U, void* stream);

/* Higher slip modes of the minimal truncation (section IV), each a fixed source that keeps its
   one-body traction (as the rank-3 trace mode d does): the septlet mode gamma and the vortlet mode
   psi (irreducible parts of the quadratic surface-velocity coefficient V^(3)) and the spinlet mode
   lambda (rank-3 part of the cubic coefficient V^(4)). With n the unit normal of the sphere, its
   surface velocity gains
       gamma: (a^2/2) gamma : n n       psi: -(a^2/3) n x (psi . n)       lambda: -(a^3/8) n x (lambda : n n)
   (the weights 1/6 and 1/90 of the surface expansion times the embeddings of the irreducible parts).
   A lone sphere does not move with them (the surface means of the slip and of n x slip vanish);
   they act on the other spheres through their exterior flows (the septlet flow is
   (7a^5/48)(1 + a^2/14 nabla^2) grad grad G : gamma, the two others are rotational, decaying as
   r^-3 and r^-4): through the strain in the right-hand side of the stresslet rows and directly in
   V and Omega.
     gam, lam [n x 10]  symmetric rank-3 tensors by the components xxx xxy xxz xyy xyz xzz yyy yyz yzz
                        zzz; only their symmetric traceless part is used
     psi      [n x 5]   symmetric traceless rank-2 tensor in the 5-basis
   Any pointer may be NULL (= zero); a NULL mbs_slip_ex* means all three are zero. */
typedef struct mbs_slip_ex {
  const double* gam;
  const double* psi;
  const double* lam;
} mbs_slip_ex;

/* mbs_solve, mbs_rhs, mbs_outputs and mbs_flow with the higher slip modes as well (arguments as
   there; ex as above). Each higher mode present costs one more all-pairs pass in the right-hand
   side and one in the outputs (all three share one pass). mbs_solve_batched and mbs_step do not
   take them. */
int mbs_solve_ex(mbs_ctx* ctx, int64_t n, const double* R, const double* p, const double* v1s,
                 const double* v2s, const double* v3t, const mbs_slip_ex* ex, const double* Fe,
                 const double* Te, const double* sigma0, double* V, double* W, double* S, double* Sigma,
                 mbs_stats* st, void* stream);
int mbs_rhs_ex(mbs_ctx* ctx, int64_t n, const double* R, const double* v2s, const double* v3t,
               const mbs_slip_ex* ex, const double* Fe, const double* Te, double* b, void* stream);
int mbs_outputs_ex(mbs_ctx* ctx, int64_t n, const double* R, const double* v1s, const double* v2s,
                   const double* v3t, const mbs_slip_ex* ex, const double* Fe, const double* Te,
                   const double* Sigma, double* V, double* W, double* S, void* stream);
int mbs_flow_ex(mbs_ctx* ctx, int64_t m, const double* X, int64_t n, const double* R, const double* Fe,
                const double* Te, const double* Sigma, const double* v3t, const mbs_slip_ex* ex, double* U,
                void* stream);

/* Traction ranks <= 3 (section IV, minimal truncation): the septlet, vortlet and potential-dipole
   traction modes become unknowns beside the flow stresslet. Each sphere's exterior flow is written
   through its flow stresslet Sigma and the equivalent slips X^gam, X^psi, X^d of the three modes
   (the slips a lone sphere would need to produce the same exterior flow of that mode; their flows
   are those of gamma, psi and d above). The Galerkin conditions of the quadratic surface modes
   (coefficient V^(3) of the incident flow, section III, split into its irreducible parts as in
   section IV: gamma its symmetric traceless part, d the contraction of the velocity index with the
   first harmonic index, psi minus the symmetric contraction with eps over those two indices) read
       X^alpha_n + P^alpha[sum_{m != n} u_m](R_n) = v^alpha_n     (alpha = gam, psi, d)
   with v^alpha_n the prescribed slip of that mode, and the stresslet rows keep their form with the
   three modes' flows among the coupled sources:
       Sigma_n / gamma - E[sum_{m != n} u_m(Sigma, X)](R_n) = E[sum_m u_m(F, T, lambda)](R_n) - c s_n.
   The spinlet mode lambda stays a fixed source (it belongs to the cubic surface coefficient).
   Unknowns, x [n x 20] row-major, per sphere:
       x[0..4]   Sigma in the 5-basis
       x[5..11]  X^gam in the 7-basis below
       x[12..16] X^psi in the 5-basis
       x[17..19] X^d (Cartesian)
   7-basis of symmetric traceless rank-3 tensors: B_m = T_m / |T_m| (Frobenius norm over all 27
   components), T_m,ijk = (1/6) d_i d_j d_k p_m for the harmonic cubics
       p_1 = 2z^3 - 3x^2 z - 3y^2 z,  p_2 = 4xz^2 - x^3 - xy^2,  p_3 = 4yz^2 - x^2 y - y^3,
       p_4 = x^2 z - y^2 z,  p_5 = xyz,  p_6 = x^3 - 3xy^2,  p_7 = 3x^2 y - y^3
   (orthonormal; coordinates x_m = B_m : T of a symmetric traceless T).
   Prescribed slips: v3t [n x 3] is v^d; ex->gam [n x 10] (symmetric components as above, traceless
   part used) is v^gam; ex->psi [n x 5] is v^psi; ex->lam [n x 10] the spinlet slip (fixed source).
   All arithmetic is binary64. Arrays are DEVICE, as elsewhere; NULL optional inputs are zero.

   mbs_matvec_r3: y [n x 20] = A x (one all-pairs pass).
   mbs_rhs_r3:    b [n x 20]: stresslet rows E[F, T, lambda] - c s; mode rows v^alpha - P^alpha[F, T,
                  lambda].
   mbs_outputs_r3: V, W [n x 3] and S [n x 5] of a solution x: V = -v1s + F/(6 pi eta a) + F^0 u,
                  W = T/(8 pi eta a^3) + (1/2) curl u over the flows u of the other spheres' F, T,
                  Sigma, X^gam, X^psi, X^d and lambda; S = Sigma + (8/3) pi eta a^3 v2s (NULL S: not
                  written).
   mbs_solve_r3:  restarted GMRES(params.restart) on A x = b to ||b - A x||_2 <= params.tol ||b||_2
                  (binary64 operator, at most params.max_iter Arnoldi steps), starting from x0
                  [n x 20], or when x0 is NULL from the one-body guess D^{-1} b (params.guess =
                  MBS_GUESS_DIAG; D as below) or zero (any other guess), then the outputs. x [n x 20]
                  (or NULL) receives the solution. With params.near_cutoff > 0 GMRES is
                  right-preconditioned by the near-field series of mbs_precond_apply_r3 (order
                  params.near_order); the solution is the same. params.precision does not apply
                  (binary64 throughout); params.check_overlap does.
   mbs_precond_apply_r3: y [n x 20] = sum_{i <= k} (-D^{-1} B_near)^i D^{-1} x, k = params.near_order,
                  with A = D + B (D = diag(I/gamma, I) per sphere, B the couplings of mbs_matvec_r3)
                  and B_near B restricted to the pairs of the near-field neighbour lists (2a <= r <
                  params.near_cutoff, at most 32 partners per sphere, the smallest indices): the
                  Neumann expansion of the inverse of the near part of the system, an addition of
                  this library (the paper names no solver). params.near_cutoff must be > 0. stats: iters, fp64_matvecs, rel_resid and
                  the timings (refinements and fp32_matvecs are 0). Returns MBS_ENOCONV (outputs of
                  the last iterate written) when the tolerance is not reached.
   Errors: MBS_EINVAL for n < 1, a missing required pointer, an output overlapping an input or
   another output, non-finite inputs (solve); MBS_EOVERLAP as mbs_solve. */
int mbs_matvec_r3(mbs_ctx* ctx, int64_t n, const double* R, const double* x, double* y, void* stream);
int mbs_rhs_r3(mbs_ctx* ctx, int64_t n, const double* R, const double* v2s, const double* v3t,
               const mbs_slip_ex* ex, const double* Fe, const double* Te, double* b, void* stream);
int mbs_outputs_r3(mbs_ctx* ctx, int64_t n, const double* R, const double* v1s, const double* v2s,
                   const mbs_slip_ex* ex, const double* Fe, const double* Te, const double* x, double* V,
                   double* W, double* S, void* stream);
int mbs_precond_apply_r3(mbs_ctx* ctx, int64_t n, const double* R, const double* x, double* y,
                         void* stream);
int mbs_solve_r3(mbs_ctx* ctx, int64_t n, const double* R, const double* v1s, const double* v2s,
                 const double* v3t, const mbs_slip_ex* ex, const double* Fe, const double* Te,
                 const double* x0, double* V, double* W, double* S, double* x, mbs_stats* st,
                 void* stream);

/* Time integration in a harmonic trap (section V set-up; kinematics of section II):
   every step rebuilds F^e = -k_trap R, T^e = 0, V^(1s) = c0 p, V^(2s) = c1 * 3(pp - I/3),
   V^(3t) = c2 p from the current state, solves, and advances
     R += dt (3/2 V_k - 1/2 V_{k-1}),  p += dt (3/2 Omega_k x p_k - 1/2 Omega_{k-1} x p_{k-1}),
   then renormalises p (order 2 = Adams-Bashforth, forward Euler on the first step; order 1 =
   forward Euler throughout). R, p [n x 3] are updated in place. slip_coef: host array [3].
   per_step: host array [nsteps] or NULL. min_dist: host array [nsteps] or NULL, receives the
   minimum centre distance of each step's configuration (overlaps are reported, not fatal).
   With params.plane the spheres must start at least a above the plane (MBS_EINVAL); each sphere's
   own image then counts as a neighbour at distance 2h (h its centre's height above the plane), so
   min_dist < 2a also reports contact with the plane; the run goes on while every centre lies
   above the plane and stops with MBS_EINVAL at the first step that finds one on or below it (R, p
   hold the state before that step).
   With params.box the distances are minimum-image ones; with params.ewald_mesh as well they come
   from the 27 neighbouring cells of a box grid (O(n); all pairs only when no pair is closer than a
   cell edge), otherwise from all pairs.
   With params.guess = MBS_GUESS_USER every step after the first starts from the previous step's
   Sigma (the first from the one-body guess). A step whose solve stops short of params.tol still
   advances and the call returns MBS_ENOCONV at the end; a non-finite residual stops the run
   (steps not taken keep zeroed per_step entries).
   hist: DEVICE [11 n] or NULL, the integrator's history (previous step's V [n x 3], Omega x p
   [n x 3], Sigma [n x 5], in that order). On return it holds the history after the last step.
   With hist_valid nonzero the call continues a run instead of starting one: the first step is an
   Adams-Bashforth step with that history and starts from that Sigma, so N steps in one call and
   N1 + N2 steps in two calls (history passed on) give identical results. */
int mbs_step(mbs_ctx* ctx, int64_t n, double* R, double* p, double k_trap, const double* slip_coef,
             double dt, int32_t nsteps, int32_t order, double* hist, int32_t hist_valid,
             mbs_stats* per_step, double* min_dist, void* stream);

/* Many independent configurations in one call (binary64 only: params.precision must be MBS_FP64,
   else MBS_EUNSUPPORTED; zero initial guess; near-field preconditioner of order params.near_order
   when params.near_cutoff > 0). Configuration b owns
   rows offsets[b] .. offsets[b+1]-1 of the concatenated device arrays (same meaning as in mbs_solve).
   offsets: HOST array [nconf + 1], offsets[0] = 0, strictly increasing. All configurations advance
   together: each pass (right-hand side, operator, Gram-Schmidt, Givens, outputs) is one launch over
   every configuration, decomposed into (configuration, receiver tile) work items, tiles of
   params.batch_item receivers or the size mbs_autotune_batched picked (largest configurations
   first); converged
   configurations drop out of later passes. A configuration is certified (binary64 residual) in the
   round of four Arnoldi steps in which its own cycle ends and then leaves the sweeps. With
   params.graph the phases are captured once per batch shape into HIP graphs on a stream owned by
   the context and replayed; from the second call of a batch shape on, the whole solve (init, the
   number of rounds the first call took, outputs) is one graph launch, followed by one read of the
   count of active configurations and more rounds only if one is still active. The call
   synchronises with `stream` on entry and exit.
   per_conf: host [nconf] or NULL (iters, rel_resid, pair_blocks, t_total_ms of the whole batch).
   latency_ms: host [nconf] or NULL: time from the start of the batch to the device clock reading
   taken when the configuration's true residual met the tolerance. Returns MBS_ENOCONV if some
   configuration did not converge (outputs are still written). */
int mbs_solve_batched(mbs_ctx* ctx, int32_t nconf, const int64_t* offsets, const double* R,
                      const double* v1s, const double* v2s, const double* v3t, const double* Fe,
                      const double* Te, double* V, double* W, double* S, double* Sigma,
                      mbs_stats* per_conf, double* latency_ms, void* stream);

/* Autotuner: time every pair-kernel launch shape of the library's candidate table (LDS-tiled
   and scalar-streamed sources, workgroup sizes, source splits) for n spheres at positions R, in
   both precisions, and use the fastest in this context (unless params.tile forces a shape).
   cache_json (may be NULL): a flat JSON object; if it holds an entry for this device and size
   class (n rounded down to a power of two) nothing is timed, otherwise the choice and its time
   are written back. chosen: host int32[2] or NULL, receives the table indices (binary64,
   binary32); params.tile = index + 1 forces that shape. */
int mbs_autotune(mbs_ctx* ctx, int64_t n, const double* R, const char* cache_json, int32_t* chosen,
                 void* stream);

/* Time the batched operator pass on this batch (offsets and R as in mbs_solve_batched) with work
   items of 64, 128 and 256 receivers, and use the fastest in this context for later
   mbs_solve_batched calls (unless params.batch_item forces a size). chosen: host int32 or NULL,
   receives the item size; ms: host double[3] or NULL, receives the average pass time of each
   candidate. The call synchronises with `stream`. */
int mbs_autotune_batched(mbs_ctx* ctx, int32_t nconf, const int64_t* offsets, const double* R,
                         int32_t* chosen, double* ms, void* stream);

/* ---------------------------------------------------------------- learned warm start
   A 3-layer perceptron in -> 128 -> 128 -> 5 (ReLU) maps the neighbourhood of each sphere to a
   correction of the one-body guess: MBS_GUESS_LEARNED starts GMRES from Sigma^0 = gamma b + net(f).
   The network multiplies bfloat16 operands with float32 accumulation on the matrix cores; its
   float32 master parameters live in the context. Its input is one of two feature sets, chosen per
   context with mbs_warmstart_features:
     MBS_FEATURES_GEOMETRY (default): in = 80, the neighbourhood geometry (see mbs_features);
     MBS_FEATURES_GEOMETRY_RHS: in = 160, each neighbour's five geometric features followed by its
       one-body stresslet gamma b_j (the diagonal solve of its stresslet row, 5 values): the part
       of the exact correction that the geometry alone cannot know (to first order the correction
       is gamma^2 sum_j K(R_i - R_j) b_j).
   Parameter vector (host float32, MBS_MLP_NPARAM or MBS_MLP_NPARAM_RHS values): W1 [in x 128]
   row-major (input x output), b1 [128], W2 [128 x 128], b2 [128], W3 [128 x 5], b3 [5]. */
#define MBS_MLP_NPARAM 27525
#define MBS_MLP_NFEAT 80
#define MBS_MLP_NPARAM_RHS 37765
#define MBS_MLP_NFEAT_RHS 160
#define MBS_FEATURES_GEOMETRY      0
#define MBS_FEATURES_GEOMETRY_RHS  1

/* Select the network's input feature set (MBS_FEATURES_*). The context's network is discarded
   (MBS_GUESS_LEARNED and the mbs_warmstart_* calls that need one fail until it is initialised, set
   or loaded again); mbs_warmstart_load selects the set the file was written with. */
int mbs_warmstart_features(mbs_ctx* ctx, int32_t feature_set);

/* Features of the warm start: for each sphere i the 16 nearest other centres j (by distance,
   ties by smaller index), nearest first, each contributing (R_j - R_i)/|R_j - R_i| (3 values),
   1/|R_j - R_i| and p_j . p_i: feat [n x 80] float32 DEVICE. nbr (may be NULL): int32 [n x 16]
   DEVICE receives the neighbour indices. Requires n >= 17. */
int mbs_features(mbs_ctx* ctx, int64_t n, const double* R, const double* p, float* feat, int32_t* nbr,
                 void* stream);
/* The features of the context's feature set: as mbs_features for MBS_FEATURES_GEOMETRY; for
   MBS_FEATURES_GEOMETRY_RHS feat [n x 160], per neighbour the five values above and then gamma b_j,
   where b [n x 5] binary64 DEVICE is the right-hand side of the same spheres (mbs_rhs; required for
   that set, else ignored). */
int mbs_features_ex(mbs_ctx* ctx, int64_t n, const double* R, const double* p, const double* b, float* feat,
                    int32_t* nbr, void* stream);
/* Initialise the network: He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)) from a 64-bit
   Mersenne twister seeded with `seed`, zero biases; resets the Adam state. */
int mbs_warmstart_init(mbs_ctx* ctx, uint64_t seed);
/* Replace / read the parameters (host float32, MBS_MLP_NPARAM or MBS_MLP_NPARAM_RHS values as the
   context's feature set); set resets the Adam state. */
int mbs_warmstart_set(mbs_ctx* ctx, const float* params);
int mbs_warmstart_get(mbs_ctx* ctx, float* params);
/* out [m x 5] = net(feat [m x in]), in = 80 or 160 as the feature set; float32 DEVICE arrays. */
int mbs_warmstart_forward(mbs_ctx* ctx, int64_t m, const float* feat, float* out, void* stream);
/* Mean squared error L = sum (net(f) - t)^2 / (5 m) over m <= 65536 samples (feat [m x in],
   target [m x 5], float32 DEVICE) and its gradient (host float32, one value per parameter, layout as the
   parameters); *loss (may be NULL) receives L. */
int mbs_warmstart_grad(mbs_ctx* ctx, int64_t m, const float* feat, const float* target, float* grad,
                       double* loss, void* stream);
/* Adam training (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) over `epochs` passes of the m
   samples in mini-batches of `batch` (16..65536), reshuffled every epoch by a Fisher-Yates
   permutation from a 64-bit Mersenne twister seeded with `seed`. loss_hist: host [epochs] or NULL,
   receives the mean training loss of each epoch. */
int mbs_warmstart_train(mbs_ctx* ctx, int64_t m, const float* feat, const float* target, int32_t epochs,
                        int32_t batch, double lr, uint64_t seed, double* loss_hist, void* stream);
/* Training target of the network for a converged flow stresslet Sigma [n x 5] (binary64 DEVICE):
   target = Sigma - gamma b as float32 [n x 5] DEVICE, b the right-hand side of the same inputs
   (arguments as in mbs_rhs). */
int mbs_warmstart_target(mbs_ctx* ctx, int64_t n, const double* R, const double* v2s, const double* v3t,
                         const double* Fe, const double* Te, const double* Sigma, float* target,
                         void* stream);
/* The initial iterate the solver would start from (sigma0 [n x 5] binary64 DEVICE) for
   guess = MBS_GUESS_ZERO (0), MBS_GUESS_DIAG (gamma b) or MBS_GUESS_LEARNED (gamma b + net). */
int mbs_initial_guess(mbs_ctx* ctx, int64_t n, const double* R, const double* p, const double* v2s,
                      const double* v3t, const double* Fe, const double* Te, int32_t guess,
                      double* sigma0, void* stream);
/* Write / read the float32 parameters (binary, little-endian uint32 header "MBSW", version 2, count,
   feature set, then the values; version 1 files (no feature set) hold 80-input networks). Loading
   selects the file's feature set in the context. */
int mbs_warmstart_save(mbs_ctx* ctx, const char* path);
int mbs_warmstart_load(mbs_ctx* ctx, const char* path);

#ifdef __cplusplus
}
#endif
#endif /* MBSTOKES_H */
