// Internal declarations shared by the kernel and host translation units of libmbstokes.
// Not part of the public interface (include/mbstokes.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace mbs {

// Physical constants of one problem, derived once on the host.
struct Phys {
  double eta, a;
  double P;          // 1 / (8 pi eta): prefactor of the Green's function flows
  double a2;         // a^2
  double a5_10;      // a^5 / 10: strength of the rank-3 trace mode flow
  double gamma;      // (20/3) pi eta a^3: lone-sphere stresslet per unit strain
  double inv_gamma;
  double mu_t;       // 1 / (6 pi eta a)
  double mu_r;       // 1 / (8 pi eta a^3)
  double slip_S;     // (8/3) pi eta a^3: traction stresslet minus flow stresslet, per unit slip
  double c_slip;     // self-slip coefficient c
};
Phys make_phys(double eta, double a, double c);

// Pair-kernel launch shape.
struct Tile {
  int variant;  // 0: sources staged through LDS tiles; 1: sources streamed by scalar (SGPR) loads
  int block;    // threads per workgroup = receivers per workgroup (64, 128 or 256)
  int tj;       // sources per LDS tile (variant 0; 64, 128 or 256)
  int wgs;      // target workgroup count used to split the sources along grid.y (0 = 2048)
};
// Candidate shapes timed by the autotuner; entry 0 is the default.
extern const Tile kTileTable[];
extern const int kTileCount;

// ---------------------------------------------------------------- pair passes
// y = x/gamma - E[x] (system operator). part: scratch [split x 5n] doubles (used when split > 1);
// src: scratch of 8n doubles (packed source records, variant 1); orig: 4 doubles of scratch.
void launch_p2(bool f32, const double* R, const double* x, double* y, double* part, double* src,
               double* orig, int64_t n, const Phys& ph, Tile t, hipStream_t s);
// y -= E* [x]: the strain of the spheres' mirror images in the plane z = plane_z (stresslet M x M,
// M = diag(1, 1, -1)) at every sphere, own image included, with the LDS kernel of tile t (the streamed
// variant falls back to 128-record tiles). part: scratch [split x 5n] as for launch_p2.
void launch_p2_image(bool f32, const double* R, const double* x, double* y, double* part, int64_t n,
                     const Phys& ph, double plane_z, Tile t, hipStream_t s);
// b = E[F, T, d] - c s
void launch_p1(const double* R, const double* v2s, const double* v3t, const double* Fe,
               const double* Te, double* b, double* part, int64_t n, const Phys& ph, Tile t,
               hipStream_t s);
// V, W, S from Sigma
void launch_p3(const double* R, const double* v1s, const double* v2s, const double* v3t,
               const double* Fe, const double* Te, const double* Sig, double* V, double* W,
               double* S, double* part, int64_t n, const Phys& ph, Tile t, hipStream_t s);
// the output pass fused with one binary64 operator application on the same Sigma:
// V, W, S as launch_p3 and y = Sigma/gamma - E[Sigma]; part: scratch [split x 11n] doubles
void launch_p23(const double* R, const double* v1s, const double* v2s, const double* v3t,
                const double* Fe, const double* Te, const double* Sig, double* y, double* V, double* W,
                double* S, double* part, int64_t n, const Phys& ph, Tile t, hipStream_t s);
// flow U [m x 3] at field points X [m x 3] from n spheres (force, torque, flow stresslet, rank-3
// trace mode; Te and v3t may be NULL); part: scratch of flow_split(m, n, t) x 3m doubles
int flow_split(int64_t m, int64_t n, Tile t);
void launch_flow(const double* X, int64_t m, const double* R, const double* Fe, const double* Te,
                 const double* Sig, const double* v3t, double* U, double* part, int64_t n, const Phys& ph,
                 Tile t, hipStream_t s);
// Septlet, vortlet and spinlet slip modes of the minimal truncation (fixed sources): gam and lam
// [n x 10] symmetric rank-3 components (traceless part used), psi [n x 5] 5-basis; NULL = absent.
struct HighSlip {
  const double* gam;
  const double* psi;
  const double* lam;
};
int high_mask(const HighSlip& h);  // bit 0 gam, bit 1 psi, bit 2 lam
// One all-pairs pass of the higher modes' sources R [n x 3] at receivers X [m x 3], added into the
// caller's arrays: target 0 strain (a [m x 5] += E), 1 rigid-body motion (a [m x 3] += U,
// b [m x 3] += W), 2 flow at field points (a [m x 3] += u). part: scratch of split x 6m doubles.
int high_split(int64_t m, int64_t n, Tile t);
void launch_high(int target, const double* X, int64_t m, const double* R, int64_t n, const HighSlip& h,
                 double* a, double* b, double* part, int split, const Phys& ph, Tile t, hipStream_t s);
// Traction ranks <= 3: one all-pairs pass over the 20 unknowns per sphere x [n x 20] = [Sigma (5-basis),
// X^gam (7-basis), X^psi (5-basis), X^d (3)]. mode 0: out = A x (out [n x 20]); mode 1: out = b from
// the fixed sources (Fe, Te, lam; NULL = absent) and the prescribed slips (v2s, gam [n x 10], psi
// [n x 5], v3t); mode 2: out = V, out2 = W [n x 3] of the solution x with the fixed sources, and
// out3 = S [n x 5] (Sigma + slip_S v2s; skipped when NULL). part: scratch of rank3_part_elems(n) doubles.
int rank3_split(int64_t n);
int64_t rank3_part_elems(int64_t n);
void launch_rank3(int mode, const double* R, const double* X20, const double* v1s, const double* v2s,
                  const double* v3t, const double* gam, const double* psi, const double* lam, const double* Fe,
                  const double* Te, double* out, double* out2, double* out3, double* part, int64_t n,
                  const Phys& ph, hipStream_t s);
// x [n x 20] = D^{-1} b, D = diag(I/gamma, I) per sphere (the one-body guess of the rank <= 3 system)
void launch_rank3_diag(const double* b, int64_t n, double gamma, double* x, hipStream_t s);
// One term of the rank <= 3 near-field Neumann series: y = D^{-1} (v - B_near z), D = diag(I/gamma,
// I), B_near the couplings of the listed pairs (launch_near_build); z == NULL stands for D^{-1} v.
// v, z, y [n x 20]; y must not overlap v or z.
void launch_rank3_near(const double* R, const double* v, const double* z, const int* cnt, const int* list,
                       int64_t n, const Phys& ph, double* y, hipStream_t s);
// Spheres above a plane z = plane_z, kind 1 stress-free (mirror images; the operator's image part
// is launch_p2_image) or kind 2 no-slip (Blake's image system, binary64): the image passes (every
// sphere's own image included). part: scratch of image_part_elems(m, n) doubles.
int image_split(int64_t m, int64_t n);
int64_t image_part_elems(int64_t m, int64_t n);
// y -= E[wall images of the stresslets x] (kind 2: the operator's image part)
void launch_wall_op(const double* R, const double* x, double* y, double* part, int64_t n, const Phys& ph,
                    double plane_z, hipStream_t s);
// b += E[images of F, T, d] (NULL = absent)
void launch_image_rhs(int kind, const double* R, const double* Fe, const double* Te, const double* v3t, double* b,
                      double* part, int64_t n, const Phys& ph, double plane_z, hipStream_t s);
// V += U, W += W of the images of F, T, Sigma, d
void launch_image_out(int kind, const double* R, const double* Fe, const double* Te, const double* Sig,
                      const double* v3t, double* V, double* W, double* part, int64_t n, const Phys& ph, double plane_z,
                      hipStream_t s);
// U [m x 3] += flow of the images at field points X [m x 3]
void launch_image_flow(int kind, const double* X, int64_t m, const double* R, int64_t n, const double* Fe,
                       const double* Te, const double* Sig, const double* v3t, double* U, double* part, const Phys& ph,
                       double plane_z, hipStream_t s);
// Spheres in a periodic cubic box of side L: Ewald summation (real space within rc <= L/2, the K
// half-lattice wave vectors kv [K x 3] on the device, 0 < |k| <= kmax). part: scratch of
// per_part_elems(n, K) doubles. Each pass writes its output completely: the operator
// y = x/gamma - E_per[x], the right-hand side b = E_per[F, T, d] - c s, the outputs V, W, S.
struct PerBox {
  double L, xi, rc;
  int K;
  const double* kv;
  const int2* seg8;  // row segments of at most 8 (operator) and 4 (other passes) wave vectors
  int nseg8;
  const int2* seg4;
  int nseg4;
  // smooth particle-mesh Ewald when M > 0: the Fourier part on an M^3 mesh (M a power of 2)
  int M;
  int nc;             // cells per axis of the sources' box grid
  const double* tab;  // pm_tables(M) on the device
  void* mws;          // pm_ws_bytes(M, n, nc) bytes of device workspace (256-byte aligned)
  const double* rtab; // the operator's radial functions tabulated for the real-space pass (npiece > 0)
  int npiece;
  void* fws;          // the flow's field-point box grid: pm_flow_ws_bytes(m, nc) bytes, or NULL (all pairs)
  size_t fws_bytes;
};
size_t pm_flow_ws_bytes(int64_t m, int nc);
// pieces of the radial table for spheres of radius^2 a2 and cutoff rc (0: no table); device doubles
// to hold any table; the table of splitting xi built on stream s
int pm_radial_pieces(double a2, double rc);
size_t pm_radial_doubles();
hipError_t pm_radial_table(double xi, double a2, double rc, double* tab, hipStream_t s);
// mesh workspace bytes for n sources; the mesh's twiddles and B-spline factors (3M doubles)
size_t pm_ws_bytes(int M, int64_t n, int nc);
std::vector<double> pm_tables(int M);
std::vector<double> per_kvecs(double L, double kmax);
// (first wave vector, count) pairs: runs of consecutive k3 within one (k1, k2) row, at most maxlen
std::vector<int> per_segments(const std::vector<double>& kv, double L, int maxlen);
// scratch doubles of one pass for m receivers and n sources with nseg structure-factor segments
// (the larger segment count)
int64_t per_part_elems(int64_t m, int64_t n, int K, int nseg);
// out[0] = the smallest minimum-image centre distance of the n >= 2 spheres; part: per_min_dist_part(n)
// doubles of scratch
int per_min_dist_part(int64_t n);
void launch_per_min_dist(const double* R, int64_t n, double L, double* part, double* out, hipStream_t s);
// the same from the box grid of a mesh box (g.M > 0, g.nc >= 3), all pairs only when no pair is closer
// than a cell edge; part: 2 per_min_dist_part(n) doubles of scratch
void launch_pm_min_dist(const double* R, int64_t n, const PerBox& g, double* part, double* out, hipStream_t s);
// U [m x 3] = flow of the periodic suspension at field points X [m x 3]
void launch_per_flow(const double* X, int64_t m, const double* R, int64_t n, const double* Fe, const double* Te,
                     const double* Sig, const double* v3t, double* U, double* part, const PerBox& g, const Phys& ph,
                     hipStream_t s);
void launch_per_op(const double* R, const double* x, double* y, double* part, int64_t n, const PerBox& g,
                   const Phys& ph, hipStream_t s);
void launch_per_rhs(const double* R, const double* v2s, const double* v3t, const double* Fe, const double* Te,
                    double* b, double* part, int64_t n, const PerBox& g, const Phys& ph, hipStream_t s);
void launch_per_out(const double* R, const double* v1s, const double* v2s, const double* v3t, const double* Fe,
                    const double* Te, const double* Sig, double* V, double* W, double* S, double* part, int64_t n,
                    const PerBox& g, const Phys& ph, hipStream_t s);
// out[0] = min over the n centres of z - plane_z (non-finite heights give -infinity)
void launch_min_height(const double* R, int64_t n, double plane_z, double* out, hipStream_t s);
// rows of R [n x 3] with z < zmin (or non-finite) -> atomically added to *cnt
void launch_count_below(const double* R, int64_t n, double zmin, int* cnt, hipStream_t s);
// min over pairs of |R_n - R_m|^2 -> out[0] (device), from the cell grid g of R (exact: an
// all-pairs scan takes over when no pair is closer than one cell edge); scratch: ceil(n/256) doubles
struct GridView;
void launch_min_dist2(const GridView& g, const double* R, int64_t n, double* out, double* scratch,
                      hipStream_t s);
// count non-finite entries of a device array -> atomically added to *cnt (device int)
void launch_count_nonfinite(const double* a, int64_t len, int* cnt, hipStream_t s);
// count rows of p [n x 3] with | |p| - 1 | > tol (or non-finite) -> atomically added to *cnt
void launch_count_nonunit(const double* p, int64_t n, double tol, int* cnt, hipStream_t s);

// near-field preconditioner: neighbour lists within rc (at most kNearCap per sphere) and
// y = gamma sum_{i <= order} (gamma K_near)^i x (order >= 2 needs tmp of 10n doubles; order 1 or
// tmp == NULL: y = gamma x + gamma^2 K_near x)
constexpr int kNearCap = 32;
// (lists from a cell grid of the centres with cell edge >= rc)
struct GridView;
void launch_near_build(const GridView& g, const double* R, double rmin, double rc, int* cnt, int* list,
                       hipStream_t s);
// (x = x + kdev[0] * ld when kdev is given)
void launch_near_apply(const double* R, const double* x, const int* cnt, const int* list, int64_t n,
                       const Phys& ph, double* y, hipStream_t s, const int* kdev = nullptr, int64_t ld = 0,
                       double* tmp = nullptr, int order = 2);

int tile_block(Tile t);                      // receivers per workgroup actually used
int split_for(int64_t n, Tile t, int tj);    // number of source chunks actually used
int64_t part_elems_max(int64_t n);           // scratch size (doubles) covering every pass and shape

// ---------------------------------------------------------------- Krylov helpers (all deterministic)
// out[k] = <V_k, w> for k < nv, V_k = V + k*ld; scratch: part [nv x dot_blocks(len)]
int dot_blocks(int64_t len);
void launch_dots(const double* V, int64_t ld, int nv, const double* w, int64_t len, double* part,
                 double* out, hipStream_t s);
// w += sign * sum_k h[k] V_k
void launch_axpy_multi(const double* V, int64_t ld, int nv, const double* h, double sign, double* w,
                       int64_t len, hipStream_t s);
// y = alpha_dev[0]^{pow} * x  with pow = -1 (divide) or +1; alpha from device memory
void launch_scale_by(const double* x, const double* alpha, int inv, double* y, int64_t len,
                     hipStream_t s);
// y = a*x + b*y (host scalars)
void launch_axpby(double a, const double* x, double b, double* y, int64_t len, hipStream_t s);
void launch_copy(const double* x, double* y, int64_t len, hipStream_t s);
// rows of `width` doubles: gather dst[k] = src[perm[k]], scatter dst[perm[k]] = src[k], k < n
void launch_gather_rows(const double* src, int width, const int32_t* perm, int64_t n, double* dst, hipStream_t s);
void launch_scatter_rows(const double* src, int width, const int32_t* perm, int64_t n, double* dst, hipStream_t s);
// One Arnoldi column: H(:,k) = h1 + h2, H(k+1,k) = sqrt(nsq); Givens update; status[0] = |g_{k+1}|,
// status[1] = H(k+1,k) (before rotation). Layout: H column-major [(m+1) x m], cs, sn, g [m+1].
void launch_givens(double* H, int m, int k, const double* h1, const double* h2, const double* nsq,
                   double* cs, double* sn, double* g, double* status, hipStream_t s);
// y = H(0:k,0:k)^{-1} g (upper triangular solve)
void launch_backsolve(const double* H, int m, int k, const double* g, double* y, hipStream_t s);
// g = [sqrt(nsq), 0, ...]; status[0] = sqrt(nsq)
void launch_init_g(const double* nsq, double* g, int m, double* status, hipStream_t s);

// ---------------------------------------------------------------- stepper
// Fe = -k R, v1s = c0 p, v2s = c1 (3pp - I) in 5-basis, v3t = c2 p
void launch_trap_modes(const double* R, const double* p, double k, double c0, double c1, double c2,
                       double* Fe, double* v1s, double* v2s, double* v3t, int64_t n, hipStream_t s);
// AB2 / Euler update of R and p (renormalised); Vprev/Pdprev updated to this step's rates.
void launch_ab_update(double* R, double* p, const double* V, const double* W, double* Vprev,
                      double* Pdprev, double dt, int first, int order, int64_t n, hipStream_t s);

}  // namespace mbs
