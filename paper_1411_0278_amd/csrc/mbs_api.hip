// Host side of libmbstokes: the C ABI, context and workspace management, and the device-resident
// GMRES / mixed-precision refinement / time-stepping drivers. All vectors stay in device memory;
// per Krylov step the host reads back two doubles (the Givens residual estimate and the new
// subdiagonal entry) to decide convergence and restarts.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <string>
#include <vector>

#include <mutex>
#include <random>

#include "../../include/mbstokes.h"
#include "mbs_batched.h"
#include "mbs_grid.h"
#include "mbs_internal.h"
#include "mbs_mlp.h"

using namespace mbs;

namespace {

thread_local std::string g_create_error;

struct DevBuf {
  double* p = nullptr;
  size_t cap = 0;  // elements
};

// Graphs of the Arnoldi steps k = 0..m-1 of one (size, positions, precision, workspace) key.
struct StepGraphs {
  std::vector<uintptr_t> key, seen;
  hipGraphExec_t g[64] = {};
  void reset() {
    for (auto& e : g)
      if (e) {
        (void)hipGraphExecDestroy(e);
        e = nullptr;
      }
    key.clear();
  }
};

}  // namespace

struct mbs_ctx {
  int device = 0;
  mbs_params prm{};
  Phys ph{};
  Tile tile64 = kTileTable[0];  // pair-kernel shapes in use (autotuned or forced by params.tile)
  Tile tile32 = kTileTable[0];
  int tuned64 = 0, tuned32 = 0;  // autotuner choices (indices into kTileTable)
  Tile tile_pass = Tile{0, 256, 128, 4096};  // shape of the right-hand-side and output passes
  std::string err;
  // workspace
  DevBuf V, w, r, b, xs, dlt, part, dpart, small, H, zeros, stepbuf, srcbuf, orig, near, zt, nt, stepstate;
  bool near_ready = false;  // neighbour lists of the current solve are built
  int* d_count = nullptr;  // device [2]: non-finite values, orientations off unit length
  double* h_status = nullptr;  // pinned host [4]
  hipEvent_t ev[8] = {};
  // event pairs bracketing operator applications inside a solve (harvested after each sync)
  static constexpr int kRing = 4;
  hipEvent_t opev[2 * kRing] = {};
  int op_prec[kRing] = {};
  int npend = 0;
  double t_op[2] = {0.0, 0.0};  // summed binary64 / binary32 operator time of the current call
  // warm-start network: float32 master parameters, gradient, Adam moments, bf16 weight copies,
  // activation workspace, neighbour lists and features
  bool mlp_ready = false;
  int adam_step = 0;
  int mlp_set = MBS_FEATURES_GEOMETRY;  // input features of the network (MBS_FEATURES_*)
  MlpLayout mlp_lay = mlp_layout(kMlpIn);
  DevBuf mlp_w, mlp_g, mlp_m, mlp_v, mlp_wb, mlp_ws, mlp_part, mlp_loss, mlp_idx, knn_buf;
  // cell grid of the centres behind both neighbour searches (near-field lists, nearest neighbours)
  DevBuf grid;
  // traction ranks <= 3: Krylov basis, residual and solution vectors, pass partial sums
  DevBuf r3;
  DevBuf per_kv;  // the periodic box's half-lattice wave vectors [per_K x 3]
  DevBuf per_seg;  // their row segments: 8-long then 4-long, (first, count) pairs
  int per_K = 0, per_nseg8 = 0, per_nseg4 = 0;
  double per_L = 0.0, per_kmax = 0.0;
  DevBuf per_tab;  // particle-mesh Ewald: the mesh's twiddles and B-spline factors
  DevBuf per_mws;  // particle-mesh Ewald: mesh fields, weights and the sources' box grid
  int per_tabM = 0;
  DevBuf per_rtab;  // particle-mesh Ewald: the operator's radial table for the real-space pass
  DevBuf per_fws;   // particle-mesh Ewald: the flow's field-point box grid
  int per_rt_np = 0;
  double per_rt_xi = 0.0, per_rt_a2 = 0.0, per_rt_rc = 0.0;
  // a solve in the Morton order of the centres: the permutation and the reordered inputs/outputs
  DevBuf ord;
  // single-configuration GMRES: Arnoldi steps captured as graphs (per precision), see step_graphs
  StepGraphs sgraph[2];
  hipStream_t gstream = nullptr;
  // batched solver: workspace, capture stream and the four graphs of the last batch shape
  DevBuf bat, btune;
  int bitem = 64;  // receivers per batched work item (mbs_autotune_batched's choice)
  hipStream_t bstream = nullptr;
  // graphs of the last batch shape: init, one round (Arnoldi steps + certification), outputs, and the
  // whole solve (init, bwhole_rounds rounds, outputs) once a solve of that shape has been observed
  hipGraphExec_t bgraph[4] = {nullptr, nullptr, nullptr, nullptr};
  int bwhole_rounds = 0;
  std::vector<uintptr_t> bkey;
  // descriptors of the last batch uploaded to the workspace (offsets, item size, workspace base):
  // an identical next batch reuses them instead of rebuilding and re-uploading
  std::vector<int64_t> bdesc_off;
  int bdesc_item = 0, bdesc_nitems = 0;
  const void* bdesc_ptr[3] = {nullptr, nullptr, nullptr};  // where they were uploaded
  uint64_t bdesc_gen = 0;  // bumped whenever a batch with other offsets or item size is uploaded
};

namespace {

int set_err(mbs_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c)
    c->err = buf;
  else
    g_create_error = buf;
  return code;
}

#define HIPCHK(ctx, expr)                                                                   \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return set_err((ctx), MBS_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e));      \
  } while (0)

#define CHK(expr)                 \
  do {                            \
    int _rc = (expr);             \
    if (_rc != MBS_OK) return _rc; \
  } while (0)

int ensure(mbs_ctx* c, DevBuf& b, size_t elems) {
  if (elems == 0) elems = 1;
  if (b.cap >= elems) return MBS_OK;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  hipError_t e = hipMalloc((void**)&b.p, elems * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_err(c, MBS_ENOMEM, "hipMalloc of %zu bytes failed: %s", elems * sizeof(double),
                   hipGetErrorString(e));
  }
  b.cap = elems;
  return MBS_OK;
}

int validate_params(mbs_ctx* c, const mbs_params* p) {
  if (!p) return set_err(c, MBS_EINVAL, "params is NULL");
  if (!(p->eta > 0.0) || !isfinite(p->eta)) return set_err(c, MBS_EINVAL, "eta must be > 0");
  if (!(p->a > 0.0) || !isfinite(p->a)) return set_err(c, MBS_EINVAL, "a must be > 0");
  if (!(p->tol > 0.0) || !(p->tol < 1.0)) return set_err(c, MBS_EINVAL, "tol must be in (0, 1)");
  if (!isfinite(p->self_slip_c)) return set_err(c, MBS_EINVAL, "self_slip_c must be finite");
  if (p->lmax != 2)
    return set_err(c, MBS_EUNSUPPORTED,
                   "lmax = %d: these entry points solve traction rank 2 (force, torque, stresslet); rank 3 "
                   "is solved by mbs_solve_r3",
                   p->lmax);
  if (p->max_iter < 1) return set_err(c, MBS_EINVAL, "max_iter must be >= 1");
  if (p->restart < 1 || p->restart > 64) return set_err(c, MBS_EINVAL, "restart must be in 1..64");
  if (p->precision != MBS_FP64 && p->precision != MBS_MIXED)
    return set_err(c, MBS_EINVAL, "precision must be MBS_FP64 or MBS_MIXED");
  if (p->precision == MBS_MIXED && !(p->inner_tol > 0.0 && p->inner_tol < 1.0))
    return set_err(c, MBS_EINVAL, "inner_tol must be in (0, 1)");
  if (p->guess < MBS_GUESS_ZERO || p->guess > MBS_GUESS_USER)
    return set_err(c, MBS_EINVAL, "unknown guess %d", p->guess);
  if (!(p->near_cutoff >= 0.0) || !isfinite(p->near_cutoff))
    return set_err(c, MBS_EINVAL, "near_cutoff must be finite and >= 0");
  if (p->tile < 0 || p->tile > kTileCount)
    return set_err(c, MBS_EINVAL, "tile must be in 0..%d", kTileCount);
  if (p->batch_item != 0 && p->batch_item != 64 && p->batch_item != 128 && p->batch_item != 256)
    return set_err(c, MBS_EINVAL, "batch_item must be 0, 64, 128 or 256");
  if (p->near_order != 0 && (p->near_order < 2 || p->near_order > 8 || (p->near_order & 1)))
    return set_err(c, MBS_EINVAL, "near_order must be 0 (= 2), 2, 4, 6 or 8");
  if (p->spatial_order < -1 || p->spatial_order > 1)
    return set_err(c, MBS_EINVAL, "spatial_order must be -1, 0 or 1");
  if (p->plane < 0 || p->plane > 2) return set_err(c, MBS_EINVAL, "plane must be 0, 1 or 2");
  if (p->plane && !isfinite(p->plane_z)) return set_err(c, MBS_EINVAL, "plane_z must be finite");
  if (!(p->box >= 0.0) || !isfinite(p->box)) return set_err(c, MBS_EINVAL, "box must be finite and >= 0");
  if (!(p->ewald_xi >= 0.0) || !isfinite(p->ewald_xi)) return set_err(c, MBS_EINVAL, "ewald_xi must be finite and >= 0");
  if (p->ewald_mesh != 0 && p->ewald_mesh != -1 &&
      (p->ewald_mesh < 16 || p->ewald_mesh > 512 || (p->ewald_mesh & (p->ewald_mesh - 1))))
    return set_err(c, MBS_EINVAL, "ewald_mesh must be 0, -1 or a power of 2 from 16 to 512");
  if (p->ewald_mesh && !(p->box > 0.0)) return set_err(c, MBS_EINVAL, "ewald_mesh needs a periodic box");
  if (p->box > 0.0 && p->ewald_xi > 0.0 && !p->ewald_mesh && p->ewald_xi * p->box < 13.0)
    return set_err(c, MBS_EINVAL, "ewald_xi * box must be at least 13 (real-space cutoff within box/2)");
  if (p->box > 0.0 && p->ewald_mesh && p->ewald_xi > 0.0 && p->ewald_xi * p->box < 10.0)
    return set_err(c, MBS_EINVAL, "ewald_xi * box must be at least 10 with a mesh (real-space cutoff within box/2)");
  if (p->box > 0.0 && p->plane) return set_err(c, MBS_EINVAL, "box and plane exclude each other");
  return MBS_OK;
}

void apply_tiles(mbs_ctx* c) {
  if (c->prm.tile > 0) {
    c->tile64 = c->tile32 = kTileTable[c->prm.tile - 1];
  } else {
    c->tile64 = kTileTable[c->tuned64];
    c->tile32 = kTileTable[c->tuned32];
  }
}

// Workspace for n spheres and restart m.
// the periodic box (params.box): splitting parameter, cutoffs and the wave vectors on the device
bool periodic(const mbs_ctx* c) { return c->prm.box > 0.0; }
// the mesh of params.ewald_mesh (-1: the smallest power of 2 from 16 to 512 whose spacing is at most
// 1.25 a), 0 for the direct sums
int mesh_M(const mbs_ctx* c) {
  const int m = c->prm.ewald_mesh;
  if (m != -1) return m;
  int M = 16;
  while (M < 512 && c->prm.box / M > 1.25 * c->prm.a) M *= 2;
  return M;
}
// default splitting: xi L = max(13, 13 (n/10^4)^0.15), measured to balance the real-space pass (whose
// pairs within rc fall as (xi L)^-3) against the Fourier passes (whose wave vectors grow as (xi L)^3)
// With a mesh of M points per axis the default is xi = pi M / (14 box): the splitting factor
// exp(-k^2 / 4 xi^2) at the mesh's Nyquist wave number pi M / box is then exp(-49/4) ~ 5e-6, which
// with B-splines of order 8 keeps the mesh error near 1e-6 of the Fourier part. The finite-size
// factors of the multipliers grow as (a k)^4, so on meshes finer than the spheres (spacing below
// about a/2) the error grows roughly as (xi a)^7: xi is kept at most 0.5/a there, and at least 10/box
// (the real-space cutoff within box/2).
double per_xi(const mbs_ctx* c, int64_t n) {
  if (c->prm.ewald_xi > 0.0) return c->prm.ewald_xi;
  if (c->prm.ewald_mesh)
    return std::max(10.0 / c->prm.box, std::min(M_PI * mesh_M(c) / (14.0 * c->prm.box), 0.5 / c->prm.a));
  return std::max(13.0, 13.0 * pow((double)n / 1e4, 0.15)) / c->prm.box;
}
// the real-space cutoff: 6.5/xi for the direct sums (below 1e-13 of the blocks), 5/xi with a mesh
// (below 1e-9, well under the mesh's own error); the cells of the sources' box grid at least rc
double per_rc(const mbs_ctx* c, double xi) {
  return std::min((c->prm.ewald_mesh ? 5.0 : 6.5) / xi, 0.5 * c->prm.box);
}
int per_nc(const mbs_ctx* c, double xi) {
  return std::max(1, std::min(256, (int)floor(c->prm.box / per_rc(c, xi))));
}
PerBox per_box(const mbs_ctx* c, int64_t n) {
  const double xi = per_xi(c, n);
  const int2* seg = reinterpret_cast<const int2*>(c->per_seg.p);
  return PerBox{c->prm.box, xi, per_rc(c, xi), c->per_K, c->per_kv.p, seg, c->per_nseg8,
                seg ? seg + c->per_nseg8 : nullptr, c->per_nseg4, mesh_M(c), per_nc(c, xi),
                c->per_tab.p, c->per_mws.p, c->per_rtab.p, c->prm.ewald_mesh ? c->per_rt_np : 0, nullptr, 0};
}
// the mesh's tables and workspace for n sources (particle-mesh Ewald)
int pm_prepare(mbs_ctx* c, int64_t n) {
  const int M = mesh_M(c);
  if (c->per_tabM != M || !c->per_tab.p) {
    const std::vector<double> t = pm_tables(M);
    CHK(ensure(c, c->per_tab, t.size()));
    HIPCHK(c, hipMemcpy(c->per_tab.p, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
    c->per_tabM = M;
  }
  const size_t bytes = pm_ws_bytes(M, n, per_nc(c, per_xi(c, n)));
  CHK(ensure(c, c->per_mws, (bytes + 7) / 8));
  const double xi = per_xi(c, n), rc = per_rc(c, xi);
  if (!c->per_rtab.p || c->per_rt_xi != xi || c->per_rt_a2 != c->ph.a2 || c->per_rt_rc != rc) {
    CHK(ensure(c, c->per_rtab, pm_radial_doubles()));
    HIPCHK(c, pm_radial_table(xi, c->ph.a2, rc, c->per_rtab.p, nullptr));
    HIPCHK(c, hipDeviceSynchronize());
    c->per_rt_np = pm_radial_pieces(c->ph.a2, rc);
    c->per_rt_xi = xi;
    c->per_rt_a2 = c->ph.a2;
    c->per_rt_rc = rc;
  }
  return MBS_OK;
}
// (re)builds the wave-vector list when the box or the splitting changed (outside any graph capture)
int per_prepare(mbs_ctx* c, int64_t n) {
  if (c->prm.ewald_mesh) return pm_prepare(c, n);
  const double kmax = 13.0 * per_xi(c, n);
  if (c->per_kv.p && c->per_L == c->prm.box && c->per_kmax == kmax) return MBS_OK;
  const std::vector<double> kv = per_kvecs(c->prm.box, kmax);
  const int K = (int)(kv.size() / 3);
  if (K < 1) return set_err(c, MBS_EINVAL, "no wave vector below the Fourier cutoff");
  CHK(ensure(c, c->per_kv, kv.size()));
  HIPCHK(c, hipMemcpy(c->per_kv.p, kv.data(), kv.size() * sizeof(double), hipMemcpyHostToDevice));
  std::vector<int> seg = per_segments(kv, c->prm.box, 8);
  const std::vector<int> seg4 = per_segments(kv, c->prm.box, 4);
  c->per_nseg8 = (int)(seg.size() / 2);
  c->per_nseg4 = (int)(seg4.size() / 2);
  seg.insert(seg.end(), seg4.begin(), seg4.end());
  CHK(ensure(c, c->per_seg, (seg.size() + 1) / 2));  // (ints stored in a double buffer)
  HIPCHK(c, hipMemcpy(c->per_seg.p, seg.data(), seg.size() * sizeof(int), hipMemcpyHostToDevice));
  c->per_K = K;
  c->per_L = c->prm.box;
  c->per_kmax = kmax;
  return MBS_OK;
}

int ensure_ws(mbs_ctx* c, int64_t n) {
  const int m = c->prm.restart;
  const int64_t len = 5 * n;
  CHK(ensure(c, c->V, (size_t)(m + 1) * len));
  CHK(ensure(c, c->w, len));
  CHK(ensure(c, c->r, len));
  CHK(ensure(c, c->b, len));
  CHK(ensure(c, c->xs, len));
  CHK(ensure(c, c->dlt, len));
  int64_t pe = std::max<int64_t>(part_elems_max(n), c->prm.plane ? image_part_elems(n, n) : 0);
  if (periodic(c)) {
    CHK(per_prepare(c, n));
    pe = std::max<int64_t>(pe, per_part_elems(n, n, c->per_K, c->per_nseg8));
  }
  CHK(ensure(c, c->part, (size_t)pe));
  CHK(ensure(c, c->srcbuf, (size_t)8 * n));
  CHK(ensure(c, c->orig, 4));
  CHK(ensure(c, c->zt, len));
  if (c->prm.near_cutoff > 0.0) {
    CHK(ensure(c, c->near, (size_t)(kNearCap + 1) * n / 2 + 64));
    CHK(ensure(c, c->nt, 2 * len));  // the preconditioner's two partial sums
  }
  CHK(ensure(c, c->dpart, (size_t)std::max<int64_t>((int64_t)(m + 2) * 256, 1024 + 2 * ((n + 255) / 256)) + 64));
  CHK(ensure(c, c->small, (size_t)8 * (m + 2) + 64));
  CHK(ensure(c, c->H, (size_t)(m + 1) * (m + 1)));
  if (c->zeros.cap < (size_t)len) {
    CHK(ensure(c, c->zeros, len));
    HIPCHK(c, hipMemset(c->zeros.p, 0, len * sizeof(double)));
  }
  return MBS_OK;
}

// small-buffer layout
struct Small {
  double *h1, *h2, *nsq, *cs, *sn, *g, *y, *status, *bnorm2;
};
Small small_of(mbs_ctx* c) {
  const int m = c->prm.restart;
  double* s = c->small.p;
  Small o;
  o.h1 = s;
  o.h2 = s + (m + 2);
  o.cs = s + 2 * (m + 2);
  o.sn = s + 3 * (m + 2);
  o.g = s + 4 * (m + 2);
  o.y = s + 5 * (m + 2);
  o.nsq = s + 6 * (m + 2);
  o.status = s + 6 * (m + 2) + 2;
  o.bnorm2 = s + 6 * (m + 2) + 6;
  return o;
}

// Accumulate the elapsed times of completed operator applications (call after a sync).
void harvest_ops(mbs_ctx* c) {
  for (int k = 0; k < c->npend; ++k) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, c->opev[2 * k], c->opev[2 * k + 1]) == hipSuccess)
      c->t_op[c->op_prec[k] == MBS_FP64 ? 0 : 1] += t;
  }
  c->npend = 0;
}

int read_status(mbs_ctx* c, const double* dev, int count, hipStream_t s) {
  HIPCHK(c, hipMemcpyAsync(c->h_status, dev, count * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  harvest_ops(c);
  return MBS_OK;
}

struct Counters {
  int iters = 0, f64 = 0, f32 = 0, refinements = 0;
  double pairs = 0.0;
};

// Arguments of the output pass, carried into the solver so that a residual expected to be the
// final one can be evaluated by the fused output + operator pass; valid: V, W, S hold the outputs
// of the current iterate.
struct OutPass {
  const double *v1s, *v2s, *v3t, *Fe, *Te;
  double *V, *W, *S;
  bool valid = false;
};

void apply_op(mbs_ctx* c, int prec, int64_t n, const double* R, const double* x, double* y,
              hipStream_t s, Counters& cnt, bool timed = true) {
  int slot = -1;
  if (timed) {  // (not inside a graph capture)
    if (c->npend == mbs_ctx::kRing) {
      (void)hipStreamSynchronize(s);
      harvest_ops(c);
    }
    slot = c->npend++;
    c->op_prec[slot] = prec;
    (void)hipEventRecord(c->opev[2 * slot], s);
  }
  if (periodic(c)) {  // the Ewald sums (binary64 in either precision)
    launch_per_op(R, x, y, c->part.p, n, per_box(c, n), c->ph, s);
    (prec == MBS_FP64 ? cnt.f64 : cnt.f32)++;
  } else if (prec == MBS_FP64) {
    launch_p2(false, R, x, y, c->part.p, c->srcbuf.p, c->orig.p, n, c->ph, c->tile64, s);
    cnt.f64++;
  } else {
    launch_p2(true, R, x, y, c->part.p, c->srcbuf.p, c->orig.p, n, c->ph, c->tile32, s);
    cnt.f32++;
  }
  if (c->prm.plane == 1) {  // the mirror images' part of the operator, in the same precision
    launch_p2_image(prec != MBS_FP64, R, x, y, c->part.p, n, c->ph, c->prm.plane_z,
                    prec == MBS_FP64 ? c->tile64 : c->tile32, s);
    cnt.pairs += (double)n * (double)n;
  } else if (c->prm.plane == 2) {  // the wall images' part (binary64 in either precision)
    launch_wall_op(R, x, y, c->part.p, n, c->ph, c->prm.plane_z, s);
    cnt.pairs += (double)n * (double)n;
  }
  if (timed) (void)hipEventRecord(c->opev[2 * slot + 1], s);
  cnt.pairs += (double)n * (double)(n - 1);
}

// y = A64 x and the outputs of x in one pass (the outputs are those of the final iterate if the
// residual formed from y passes); timed by events 4-5 of the context.
void apply_op_out(mbs_ctx* c, int64_t n, const double* R, const double* x, double* y, OutPass& o,
                  hipStream_t s, Counters& cnt) {
  (void)hipEventRecord(c->ev[4], s);
  if (periodic(c)) {  // operator and outputs as two Ewald passes
    launch_per_op(R, x, y, c->part.p, n, per_box(c, n), c->ph, s);
    launch_per_out(R, o.v1s, o.v2s, o.v3t, o.Fe, o.Te, x, o.V, o.W, o.S, c->part.p, n, per_box(c, n), c->ph, s);
    (void)hipEventRecord(c->ev[5], s);
    cnt.pairs += 2.0 * (double)n * (double)(n - 1);
    o.valid = true;
    return;
  }
  launch_p23(R, o.v1s, o.v2s, o.v3t, o.Fe, o.Te, x, y, o.V, o.W, o.S, c->part.p, n, c->ph, c->tile_pass, s);
  if (c->prm.plane) {
    if (c->prm.plane == 1)
      launch_p2_image(false, R, x, y, c->part.p, n, c->ph, c->prm.plane_z, c->tile64, s);
    else
      launch_wall_op(R, x, y, c->part.p, n, c->ph, c->prm.plane_z, s);
    launch_image_out(c->prm.plane, R, o.Fe, o.Te, x, o.v3t, o.V, o.W, c->part.p, n, c->ph, c->prm.plane_z, s);
    cnt.pairs += 2.0 * (double)n * (double)n;
  }
  (void)hipEventRecord(c->ev[5], s);
  cnt.pairs += 2.0 * (double)n * (double)(n - 1);
  o.valid = true;
}

// ||v||^2 into dev[0]
void norm2(mbs_ctx* c, const double* v, int64_t len, double* dev, hipStream_t s) {
  launch_dots(v, 0, 1, v, len, c->dpart.p, dev, s);
}

// Restarted GMRES on A x = rhs, operator precision prec. x is updated in place (x_zero: x is 0).
// Stops when the residual estimate is <= tol_abs. With verify, the final residual is recomputed
// with the operator and returned in *resid; otherwise *resid is the last estimate.
// near-field preconditioner lists for the current positions
// cell grid of R with cell edge >= h_min and at most max_cells cells, in the context's workspace
int grid_of(mbs_ctx* c, int64_t n, const double* R, double h_min, int64_t max_cells, GridView* g,
            hipStream_t s) {
  const size_t bytes = grid_ws_bytes((int)n, max_cells);
  CHK(ensure(c, c->grid, bytes / 8 + 64));
  HIPCHK(c, grid_build(R, (int)n, h_min, max_cells, c->grid.p, c->grid.cap * 8, g, s));
  return MBS_OK;
}

// near-field preconditioner lists for the current positions (grid cells of edge >= r_c, at most
// about two cells per sphere)
int near_prepare(mbs_ctx* c, int64_t n, const double* R, hipStream_t s) {
  GridView g;
  CHK(grid_of(c, n, R, c->prm.near_cutoff, 2 * n + 64, &g, s));
  int* cntp = (int*)c->near.p;
  launch_near_build(g, R, 2.0 * c->prm.a, c->prm.near_cutoff, cntp, cntp + n, s);
  HIPCHK(c, hipGetLastError());
  c->near_ready = true;
  return MBS_OK;
}
int near_order(const mbs_ctx* c) { return c->prm.near_order ? c->prm.near_order : 2; }
void near_apply(mbs_ctx* c, int64_t n, const double* R, const double* x, double* y, hipStream_t s) {
  const int* cntp = (const int*)c->near.p;
  launch_near_apply(R, x, cntp, cntp + n, n, c->ph, y, s, nullptr, 0, c->nt.p, near_order(c));
}

// Small systems are bound by launch and synchronisation latency, so their Arnoldi steps are
// captured into graphs (one per step index k, the kernels' pointers and sizes fixed) and replayed.
// A key seen for the first time runs eagerly; from its second use (the stepper, repeated solves of
// one configuration) the steps are captured once and replayed. Any change of size, positions
// pointer, precision, preconditioning, launch shape or workspace drops the graphs.
constexpr int64_t kGraphMaxN = 32768;

uintptr_t dbits(double v) {
  uintptr_t b = 0;
  memcpy(&b, &v, sizeof(v) < sizeof(b) ? sizeof(v) : sizeof(b));
  return b;
}

StepGraphs* step_graphs(mbs_ctx* c, int prec, int64_t n, const double* R, bool pc) {
  if (!c->prm.graph || n > kGraphMaxN) return nullptr;
  const Tile t = prec == MBS_FP64 ? c->tile64 : c->tile32;
  const std::vector<uintptr_t> key = {
      (uintptr_t)n, (uintptr_t)R, (uintptr_t)pc, (uintptr_t)t.variant, (uintptr_t)t.block, (uintptr_t)t.tj,
      (uintptr_t)t.wgs, (uintptr_t)c->prm.restart, (uintptr_t)c->V.p, (uintptr_t)c->w.p, (uintptr_t)c->zt.p, (uintptr_t)c->nt.p,
      (uintptr_t)c->H.p, (uintptr_t)c->small.p, (uintptr_t)c->dpart.p, (uintptr_t)c->part.p,
      (uintptr_t)c->srcbuf.p, (uintptr_t)c->orig.p, (uintptr_t)c->near.p, (uintptr_t)near_order(c),
      dbits(c->ph.P), dbits(c->ph.a2),
      dbits(c->ph.gamma), dbits(c->ph.inv_gamma), (uintptr_t)c->prm.plane, dbits(c->prm.plane_z),
      dbits(c->prm.box), dbits(c->prm.ewald_xi), (uintptr_t)c->per_kv.p, (uintptr_t)c->per_K,
      (uintptr_t)c->per_seg.p, (uintptr_t)c->per_nseg8, (uintptr_t)mesh_M(c), (uintptr_t)c->per_tab.p,
      (uintptr_t)c->per_mws.p};
  StepGraphs& G = c->sgraph[prec == MBS_FP64 ? 0 : 1];
  if (key == G.key) return &G;
  G.reset();
  if (key == G.seen) {
    G.key = key;
    return &G;
  }
  G.seen = key;
  return nullptr;
}

// Launch Arnoldi step k from its graph, capturing it first if needed (on a stream of the context).
template <typename Fn>
int launch_step_graph(mbs_ctx* c, StepGraphs& G, int k, Fn enqueue, hipStream_t s) {
  if (!G.g[k]) {
    if (!c->gstream) HIPCHK(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
    enqueue(c->gstream);
    HIPCHK(c, hipStreamEndCapture(c->gstream, &g));
    hipError_t e = hipGraphInstantiate(&G.g[k], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      G.g[k] = nullptr;
      return set_err(c, MBS_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
  }
  HIPCHK(c, hipGraphLaunch(G.g[k], s));
  return MBS_OK;
}

int gmres(mbs_ctx* c, int prec, int64_t n, const double* R, const double* rhs, double* x,
          bool x_zero, double tol_abs, int max_iters, bool verify, double* resid, Counters& cnt,
          hipStream_t s, OutPass* out = nullptr) {
  const int m = c->prm.restart;
  const bool pc = c->prm.near_cutoff > 0.0 && c->near_ready;  // right preconditioning: A M^{-1} u = r
  const int64_t len = 5 * n;
  Small sm = small_of(c);
  double* V = c->V.p;
  double* w = c->w.p;
  double* r = c->r.p;
  StepGraphs* sg = step_graphs(c, prec, n, R, pc);
  // initial residual
  if (x_zero) {
    launch_copy(rhs, r, len, s);
  } else {
    apply_op(c, prec, n, R, x, r, s, cnt);
    launch_axpby(1.0, rhs, -1.0, r, len, s);
  }
  norm2(c, r, len, sm.nsq, s);
  launch_init_g(sm.nsq, sm.g, m, sm.status, s);
  CHK(read_status(c, sm.status, 1, s));
  double beta = c->h_status[0];
  int used = 0;
  while (beta > tol_abs && used < max_iters) {
    launch_scale_by(r, sm.status, 1, V, len, s);  // V0 = r / beta (status[0] = beta)
    int k = 0;
    double est = beta;
    bool breakdown = false;
    while (k < m && used < max_iters) {
      // Arnoldi step k: w = A (M^{-1}) v_k, classical Gram-Schmidt applied twice, Givens update
      auto step = [&, k](hipStream_t q, bool timed, Counters& ct) {
        double* vk = V + (int64_t)k * len;
        if (pc) {
          near_apply(c, n, R, vk, c->zt.p, q);
          apply_op(c, prec, n, R, c->zt.p, w, q, ct, timed);
        } else {
          apply_op(c, prec, n, R, vk, w, q, ct, timed);
        }
        launch_dots(V, len, k + 1, w, len, c->dpart.p, sm.h1, q);
        launch_axpy_multi(V, len, k + 1, sm.h1, -1.0, w, len, q);
        launch_dots(V, len, k + 1, w, len, c->dpart.p, sm.h2, q);
        launch_axpy_multi(V, len, k + 1, sm.h2, -1.0, w, len, q);
        norm2(c, w, len, sm.nsq, q);
        launch_givens(c->H.p, m, k, sm.h1, sm.h2, sm.nsq, sm.cs, sm.sn, sm.g, sm.status, q);
        launch_scale_by(w, sm.status + 1, 1, V + (int64_t)(k + 1) * len, len, q);
      };
      if (sg) {
        Counters scratch;  // the capture's own counts are not the replays'
        CHK(launch_step_graph(c, *sg, k, [&](hipStream_t q) { step(q, false, scratch); }, s));
        (prec == MBS_FP64 ? cnt.f64 : cnt.f32)++;
        cnt.pairs += (double)n * (double)(n - 1);
      } else {
        step(s, true, cnt);
      }
      CHK(read_status(c, sm.status, 2, s));
      est = c->h_status[0];
      ++k;
      ++used;
      cnt.iters++;
      if (!(c->h_status[1] > 1e-300 * beta)) breakdown = true;
      if (est <= tol_abs || breakdown) break;
    }
    launch_backsolve(c->H.p, m, k, sm.g, sm.y, s);
    if (pc) {  // x += M^{-1} (V y)
      launch_axpby(0.0, w, 0.0, c->zt.p, len, s);
      launch_axpy_multi(V, len, k, sm.y, 1.0, c->zt.p, len, s);
      near_apply(c, n, R, c->zt.p, w, s);
      launch_axpby(1.0, w, 1.0, x, len, s);
    } else {
      launch_axpy_multi(V, len, k, sm.y, 1.0, x, len, s);
    }
    x_zero = false;
    const bool done = est <= tol_abs || breakdown || used >= max_iters;
    if (done && !verify) {
      beta = est;
      break;
    }
    if (done && out && prec == MBS_FP64) {
      apply_op_out(c, n, R, x, r, *out, s, cnt);  // expected final: fuse the output pass
    } else {
      apply_op(c, prec, n, R, x, r, s, cnt);
      if (out) out->valid = false;
    }
    launch_axpby(1.0, rhs, -1.0, r, len, s);
    norm2(c, r, len, sm.nsq, s);
    launch_init_g(sm.nsq, sm.g, m, sm.status, s);
    CHK(read_status(c, sm.status, 1, s));
    beta = c->h_status[0];
    if (done) break;
  }
  *resid = beta;
  return MBS_OK;
}

// Orientations must be unit vectors to this tolerance wherever they are read (the slip modes and
// the learned guess's features are built from them).
constexpr double kUnitTol = 1e-12;

// Counts, in one round trip, the non-finite values of the given arrays (*bad) and, when p is given,
// the rows of p [n x 3] whose length is not within kUnitTol of 1 (*bad_p).
int count_bad(mbs_ctx* c, hipStream_t s, std::initializer_list<std::pair<const double*, int64_t>> arrs,
              int* bad, const double* p = nullptr, int64_t n = 0, int* bad_p = nullptr) {
  HIPCHK(c, hipMemsetAsync(c->d_count, 0, 2 * sizeof(int), s));
  for (auto& a : arrs)
    if (a.first) launch_count_nonfinite(a.first, a.second, c->d_count, s);
  if (p) launch_count_nonunit(p, n, kUnitTol, c->d_count + 1, s);
  int h[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(h, c->d_count, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  *bad = h[0];
  if (bad_p) *bad_p = h[1];
  return MBS_OK;
}

int count_nonfinite(mbs_ctx* c, hipStream_t s, std::initializer_list<std::pair<const double*, int64_t>> arrs,
                    int* bad) {
  return count_bad(c, s, arrs, bad);
}

// Non-finite inputs and orientations off unit length are argument errors.
int check_inputs(mbs_ctx* c, hipStream_t s, std::initializer_list<std::pair<const double*, int64_t>> arrs,
                 const double* p, int64_t n) {
  int bad = 0, bad_p = 0;
  CHK(count_bad(c, s, arrs, &bad, p, n, &bad_p));
  if (bad) return set_err(c, MBS_EINVAL, "%d non-finite input values", bad);
  if (bad_p)
    return set_err(c, MBS_EINVAL, "%d orientations p are not unit vectors (| |p| - 1 | > %.0e)", bad_p, kUnitTol);
  return MBS_OK;
}

// With params.plane, the points X [m x 3] must lie at or above zmin (non-finite ones count as below).
int check_above(mbs_ctx* c, hipStream_t s, const double* X, int64_t m, double zmin, const char* what) {
  HIPCHK(c, hipMemsetAsync(c->d_count, 0, sizeof(int), s));
  launch_count_below(X, m, zmin, c->d_count, s);
  int h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, c->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (h) return set_err(c, MBS_EINVAL, "%d %s", h, what);
  return MBS_OK;
}
// every sphere at least a above the plane (a no-op without params.plane)
int check_plane(mbs_ctx* c, hipStream_t s, const double* R, int64_t n) {
  if (!c->prm.plane) return MBS_OK;
  return check_above(c, s, R, n, c->prm.plane_z + c->prm.a,
                     "sphere centres lie less than a above the plane (params.plane_z + a)");
}
// entry points that do not take the plane
int refuse_plane(mbs_ctx* c, const char* what) {
  if (c->prm.plane) return set_err(c, MBS_EUNSUPPORTED, "%s does not support params.plane", what);
  if (c->prm.box > 0.0) return set_err(c, MBS_EUNSUPPORTED, "%s does not support params.box", what);
  return MBS_OK;
}
// entry points that take the plane but not the periodic box
int refuse_box(mbs_ctx* c, const char* what) {
  if (c->prm.box > 0.0) return set_err(c, MBS_EUNSUPPORTED, "%s does not support params.box", what);
  return MBS_OK;
}

// An output array may not share memory with an input or with another output: the passes read their
// inputs while writing their outputs. Each entry is (name, pointer, number of doubles); NULL entries
// are skipped.
struct Span {
  const char* name;
  const void* p;
  int64_t len;
};
int check_aliasing(mbs_ctx* c, std::initializer_list<Span> outs, std::initializer_list<Span> ins) {
  auto hit = [](const Span& a, const Span& b) {
    if (!a.p || !b.p || a.len <= 0 || b.len <= 0) return false;
    const uintptr_t a0 = (uintptr_t)a.p, a1 = a0 + (uintptr_t)a.len * sizeof(double);
    const uintptr_t b0 = (uintptr_t)b.p, b1 = b0 + (uintptr_t)b.len * sizeof(double);
    return a0 < b1 && b0 < a1;
  };
  for (auto o = outs.begin(); o != outs.end(); ++o) {
    for (const Span& i : ins)
      if (hit(*o, i)) return set_err(c, MBS_EINVAL, "output %s overlaps input %s", o->name, i.name);
    for (auto q = outs.begin(); q != o; ++q)
      if (hit(*o, *q)) return set_err(c, MBS_EINVAL, "outputs %s and %s overlap", q->name, o->name);
  }
  return MBS_OK;
}

// The learned guess needs a network, the orientations and at least kNeigh other spheres.
int check_learned(mbs_ctx* c, int64_t n, const double* p) {
  if (!c->mlp_ready)
    return set_err(c, MBS_EUNSUPPORTED, "no warm-start network in this context (mbs_warmstart_*)");
  if (!p) return set_err(c, MBS_EINVAL, "the learned guess needs the orientations p");
  if (n < kNeigh + 1) return set_err(c, MBS_EINVAL, "the learned guess needs n >= %d", kNeigh + 1);
  return MBS_OK;
}

int check_overlap(mbs_ctx* c, int64_t n, const double* R, hipStream_t s, double* min_d) {
  if (n < 2) {
    *min_d = INFINITY;
    return MBS_OK;
  }
  double* out = c->small.p + c->small.cap - 1;
  GridView g;  // cells of edge >= 3a, at most about two per sphere
  CHK(grid_of(c, n, R, 3.0 * c->prm.a, 2 * n + 64, &g, s));
  launch_min_dist2(g, R, n, out, c->dpart.p + 1024, s);
  CHK(read_status(c, out, 1, s));
  *min_d = sqrt(c->h_status[0]);
  return MBS_OK;
}

// smallest minimum-image centre distance in the periodic box (params.box; infinity for one sphere)
int per_min_dist(mbs_ctx* c, int64_t n, const double* R, hipStream_t s, double* md) {
  if (n < 2) {
    *md = INFINITY;
    return MBS_OK;
  }
  // (the tail of dpart holds at least 2 (n + 255)/256 + 64 doubles beyond offset 1024)
  double* out = c->small.p + c->small.cap - 1;
  const PerBox g = per_box(c, n);
  if (g.M > 0 && g.nc >= 3)
    launch_pm_min_dist(R, n, g, c->dpart.p + 1024, out, s);
  else
    launch_per_min_dist(R, n, c->prm.box, c->dpart.p + 1024, out, s);
  CHK(read_status(c, out, 1, s));
  *md = c->h_status[0];
  return MBS_OK;
}

// lowest centre's height above the plane (params.plane)
int min_height(mbs_ctx* c, int64_t n, const double* R, hipStream_t s, double* h) {
  double* out = c->small.p + c->small.cap - 1;
  launch_min_height(R, n, c->prm.plane_z, out, s);
  CHK(read_status(c, out, 1, s));
  *h = c->h_status[0];
  return MBS_OK;
}

float ev_ms(hipEvent_t a, hipEvent_t b) {
  float t = 0.f;
  if (hipEventElapsedTime(&t, a, b) != hipSuccess) return 0.f;
  return t;
}

// ---------------------------------------------------------------- warm-start network (host side)
constexpr int kChunkRows = 65536;  // rows per network pass (bounds the activation workspace)

struct MlpWs {
  uint16_t *X, *H1, *H2, *dOut, *D2, *D1;
  float *C1, *C2, *C3, *dOut32, *G2, *G2m, *G1, *G1m;
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t mlp_ws_bytes(int rp) {
  size_t b = 0;
  b += align256((size_t)rp * kMlpInMax * 2);
  b += 2 * align256((size_t)rp * kMlpHid * 2);      // H1, H2
  b += align256((size_t)rp * 16 * 2);               // dOut
  b += 2 * align256((size_t)rp * kMlpHid * 2);      // D2, D1
  b += 2 * align256((size_t)rp * kMlpHid * 4);      // C1, C2
  b += align256((size_t)rp * 16 * 4);               // C3
  b += align256((size_t)rp * kMlpOut * 4);          // dOut32
  b += 4 * align256((size_t)rp * kMlpHid * 4);      // G2, G2m, G1, G1m
  return b;
}

int mlp_ensure(mbs_ctx* c, int rp) {
  CHK(ensure(c, c->mlp_w, (kMlpParamsMax + 1) / 2 + 8));
  CHK(ensure(c, c->mlp_g, (kMlpParamsMax + 1) / 2 + 8));
  CHK(ensure(c, c->mlp_m, (kMlpParamsMax + 1) / 2 + 8));
  CHK(ensure(c, c->mlp_v, (kMlpParamsMax + 1) / 2 + 8));
  CHK(ensure(c, c->mlp_wb, (kMlpInMax * kMlpHid + kMlpHid * kMlpHid + kMlpHid * 16) / 4 + 64));
  CHK(ensure(c, c->mlp_ws, mlp_ws_bytes(rp) / 8 + 64));
  // split-K partial products of the weight gradients: up to 64 chunks of [max(in, 128) x 128] floats
  CHK(ensure(c, c->mlp_part, (size_t)64 * std::max(kMlpInMax, kMlpHid) * kMlpHid / 2 + 64));
  CHK(ensure(c, c->mlp_loss, (size_t)mlp_mse_blocks(rp) + 64));
  return MBS_OK;
}

MlpWs mlp_carve(mbs_ctx* c, int rp) {
  char* p = (char*)c->mlp_ws.p;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += align256(bytes);
    return q;
  };
  MlpWs w;
  w.X = (uint16_t*)take((size_t)rp * kMlpInMax * 2);
  w.H1 = (uint16_t*)take((size_t)rp * kMlpHid * 2);
  w.H2 = (uint16_t*)take((size_t)rp * kMlpHid * 2);
  w.dOut = (uint16_t*)take((size_t)rp * 16 * 2);
  w.D2 = (uint16_t*)take((size_t)rp * kMlpHid * 2);
  w.D1 = (uint16_t*)take((size_t)rp * kMlpHid * 2);
  w.C1 = (float*)take((size_t)rp * kMlpHid * 4);
  w.C2 = (float*)take((size_t)rp * kMlpHid * 4);
  w.C3 = (float*)take((size_t)rp * 16 * 4);
  w.dOut32 = (float*)take((size_t)rp * kMlpOut * 4);
  w.G2 = (float*)take((size_t)rp * kMlpHid * 4);
  w.G2m = (float*)take((size_t)rp * kMlpHid * 4);
  w.G1 = (float*)take((size_t)rp * kMlpHid * 4);
  w.G1m = (float*)take((size_t)rp * kMlpHid * 4);
  return w;
}

struct MlpW {
  float* w;
  uint16_t *W1, *W2, *W3;
};
MlpW mlp_weights(mbs_ctx* c) {
  MlpW o;
  o.w = (float*)c->mlp_w.p;
  o.W1 = (uint16_t*)c->mlp_wb.p;
  o.W2 = o.W1 + kMlpInMax * kMlpHid;
  o.W3 = o.W2 + kMlpHid * kMlpHid;
  return o;
}

int ceil16(int v) { return (v + 15) & ~15; }

// forward pass of `rows` samples (feature rows idx[r] of feat, or r if idx is NULL) -> C3 [rp x 16]
void mlp_forward_rows(mbs_ctx* c, const float* feat, const int32_t* idx, int rows, const MlpWs& ws,
                      hipStream_t s) {
  const int rp = ceil16(rows);
  MlpW W = mlp_weights(c);
  const MlpLayout& L = c->mlp_lay;
  float* part = (float*)c->mlp_part.p;
  mlp_gather_bf16(feat, idx, rows, rp, L.in, ws.X, s);
  mlp_gemm(ws.X, L.in, false, W.W1, kMlpHid, false, ws.C1, part, rp, kMlpHid, L.in, 1, s);
  mlp_bias_relu(ws.C1, W.w + L.offB1, rp, kMlpHid, ws.H1, s);
  mlp_gemm(ws.H1, kMlpHid, false, W.W2, kMlpHid, false, ws.C2, part, rp, kMlpHid, kMlpHid, 1, s);
  mlp_bias_relu(ws.C2, W.w + L.offB2, rp, kMlpHid, ws.H2, s);
  mlp_gemm(ws.H2, kMlpHid, false, W.W3, 16, false, ws.C3, part, rp, 16, kMlpHid, 1, s);
}

// gradient of the batch MSE into c->mlp_g; loss partial sums into c->mlp_loss (+ loss_off)
void mlp_backward_rows(mbs_ctx* c, const float* target, const int32_t* idx, int rows,
                       const MlpWs& ws, double* loss_parts, hipStream_t s) {
  const int rp = ceil16(rows);
  MlpW W = mlp_weights(c);
  const MlpLayout& L = c->mlp_lay;
  float* g = (float*)c->mlp_g.p;
  float* part = (float*)c->mlp_part.p;
  const int ks = std::max(1, std::min(64, rp / 512));
  mlp_mse_grad(ws.C3, W.w + L.offB3, target, idx, rows, rp, 1.0 / ((double)rows * kMlpOut), ws.dOut,
               ws.dOut32, loss_parts, s);
  // W3, b3
  mlp_gemm(ws.H2, kMlpHid, true, ws.dOut, 16, false, ws.G2 /*scratch [128 x 16]*/, part, kMlpHid, 16,
           rp, ks, s);
  mlp_copy_cols(ws.G2, 16, kMlpHid, kMlpOut, g + L.offW3, s);
  mlp_colsum(ws.dOut32, rows, kMlpOut, g + L.offB3, part, s);
  // through layer 3
  mlp_gemm(ws.dOut, 16, false, W.W3, 16, true, ws.G2, part, rp, kMlpHid, 16, 1, s);
  mlp_relu_mask(ws.G2, ws.H2, (int64_t)rp * kMlpHid, ws.D2, ws.G2m, s);
  mlp_colsum(ws.G2m, rp, kMlpHid, g + L.offB2, part, s);
  mlp_gemm(ws.H1, kMlpHid, true, ws.D2, kMlpHid, false, g + L.offW2, part, kMlpHid, kMlpHid, rp, ks, s);
  // through layer 2
  mlp_gemm(ws.D2, kMlpHid, false, W.W2, kMlpHid, true, ws.G1, part, rp, kMlpHid, kMlpHid, 1, s);
  mlp_relu_mask(ws.G1, ws.H1, (int64_t)rp * kMlpHid, ws.D1, ws.G1m, s);
  mlp_colsum(ws.G1m, rp, kMlpHid, g + L.offB1, part, s);
  mlp_gemm(ws.X, L.in, true, ws.D1, kMlpHid, false, g + L.offW1, part, L.in, kMlpHid, rp, ks, s);
}

// network output for m samples: out [m x 5] float32
int mlp_forward(mbs_ctx* c, int64_t m, const float* feat, float* out, hipStream_t s) {
  const int rp_max = (int)std::min<int64_t>(ceil16((int)std::min<int64_t>(m, kChunkRows)), kChunkRows);
  CHK(mlp_ensure(c, rp_max));
  MlpWs ws = mlp_carve(c, rp_max);
  MlpW W = mlp_weights(c);
  for (int64_t r0 = 0; r0 < m; r0 += kChunkRows) {
    const int rows = (int)std::min<int64_t>(kChunkRows, m - r0);
    mlp_forward_rows(c, feat + r0 * c->mlp_lay.in, nullptr, rows, ws, s);
    mlp_out_bias(ws.C3, W.w + c->mlp_lay.offB3, rows, out + r0 * kMlpOut, s);
  }
  return MBS_OK;
}

// features of feature set `set` (MBS_FEATURES_GEOMETRY_RHS reads b, the right-hand side [n x 5])
int knn_features(mbs_ctx* c, int64_t n, const double* R, const double* p, float* feat, int32_t* nbr,
                 hipStream_t s, int set = MBS_FEATURES_GEOMETRY, const double* b = nullptr) {
  // cells of edge >= a holding about eight centres each: the 16th neighbour is usually inside the
  // 27 cells around a sphere's own
  GridView g;
  CHK(grid_of(c, n, R, c->prm.a, std::max<int64_t>(64, n / 8), &g, s));
  launch_knn16(g, nbr, s);
  if (set == MBS_FEATURES_GEOMETRY_RHS)
    launch_features(R, p, nbr, (int)n, feat, s, b, c->ph.gamma);
  else
    launch_features(R, p, nbr, (int)n, feat, s);
  HIPCHK(c, hipGetLastError());
  return MBS_OK;
}

// learned guess: x = gamma b + network(features(R, p))
int learned_guess(mbs_ctx* c, int64_t n, const double* R, const double* p, const double* b, double* x,
                  hipStream_t s) {
  const size_t o_feat = align256((size_t)n * kNeigh * 4);
  const size_t o_out = o_feat + align256((size_t)n * c->mlp_lay.in * 4);
  const size_t bytes = o_out + (size_t)n * kMlpOut * 4;
  CHK(ensure(c, c->knn_buf, bytes / 8 + 64));
  char* base = (char*)c->knn_buf.p;
  int32_t* nbr = (int32_t*)base;
  float* feat = (float*)(base + o_feat);
  float* out = (float*)(base + o_out);
  CHK(knn_features(c, n, R, p, feat, nbr, s, c->mlp_set, b));
  CHK(mlp_forward(c, n, feat, out, s));
  launch_guess_learned(b, out, c->ph.gamma, 5 * n, x, s);
  return MBS_OK;
}

// The solve without argument validation, in the order given; sigma0 is read for MBS_GUESS_USER.
int solve_in_order(mbs_ctx* c, int64_t n, const double* R, const double* p, const double* v1s, const double* v2s,
                   const double* v3t, const double* Fe, const double* Te, const HighSlip& hi, const double* sigma0,
                   double* V, double* W, double* S, double* Sigma, mbs_stats* st, hipStream_t s) {
  CHK(ensure_ws(c, n));
  const bool high = high_mask(hi) != 0;
  const int hsplit = high_split(n, n, c->tile_pass);
  const int64_t len = 5 * n;
  const double* Fz = Fe ? Fe : c->zeros.p;
  Counters cnt;
  Small sm = small_of(c);
  c->npend = 0;
  c->t_op[0] = c->t_op[1] = 0.0;
  c->near_ready = false;
  HIPCHK(c, hipEventRecord(c->ev[0], s));
  if (c->prm.superposition) {
    // superposition approximation (section IV): every sphere keeps its lone-sphere stresslet
    // Sigma_n = -c gamma s_n, no system is solved, the motion is the direct sum of the pair flows
    launch_axpby(-c->ph.c_slip * c->ph.gamma, v2s ? v2s : c->zeros.p, 0.0, c->xs.p, len, s);
    HIPCHK(c, hipEventRecord(c->ev[1], s));
    HIPCHK(c, hipEventRecord(c->ev[2], s));
    if (periodic(c))
      launch_per_out(R, v1s, v2s, v3t, Fz, Te, c->xs.p, V, W, S, c->part.p, n, per_box(c, n), c->ph, s);
    else
      launch_p3(R, v1s, v2s, v3t, Fz, Te, c->xs.p, V, W, S, c->part.p, n, c->ph, c->tile_pass, s);
    if (high) launch_high(1, R, n, R, n, hi, V, W, c->part.p, hsplit, c->ph, c->tile_pass, s);
    if (c->prm.plane)
      launch_image_out(c->prm.plane, R, Fe, Te, c->xs.p, v3t, V, W, c->part.p, n, c->ph, c->prm.plane_z, s);
    if (Sigma) launch_copy(c->xs.p, Sigma, len, s);
    HIPCHK(c, hipEventRecord(c->ev[3], s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (st) {
      memset(st, 0, sizeof(*st));
      st->t_out_ms = st->t_total_ms = ev_ms(c->ev[2], c->ev[3]);
      st->pair_blocks = (double)n * (double)(n - 1) * (high ? 2.0 : 1.0);
    }
    return MBS_OK;
  }
  if (c->prm.near_cutoff > 0.0) CHK(near_prepare(c, n, R, s));
  // right-hand side
  if (periodic(c))
    launch_per_rhs(R, v2s, v3t, Fz, Te, c->b.p, c->part.p, n, per_box(c, n), c->ph, s);
  else
    launch_p1(R, v2s, v3t, Fz, Te, c->b.p, c->part.p, n, c->ph, c->tile_pass, s);
  cnt.pairs += (double)n * (double)(n - 1);
  if (c->prm.plane) {
    launch_image_rhs(c->prm.plane, R, Fe, Te, v3t, c->b.p, c->part.p, n, c->ph, c->prm.plane_z, s);
    cnt.pairs += (double)n * (double)n;
  }
  if (high) {  // strain of the septlet, vortlet and spinlet flows
    launch_high(0, R, n, R, n, hi, c->b.p, nullptr, c->part.p, hsplit, c->ph, c->tile_pass, s);
    cnt.pairs += (double)n * (double)(n - 1);
  }
  HIPCHK(c, hipEventRecord(c->ev[1], s));
  norm2(c, c->b.p, len, sm.bnorm2, s);
  CHK(read_status(c, sm.bnorm2, 1, s));
  const double bnorm = sqrt(c->h_status[0]);
  // initial guess
  bool x_zero = false;
  switch (c->prm.guess) {
    case MBS_GUESS_ZERO:
      HIPCHK(c, hipMemsetAsync(c->xs.p, 0, len * sizeof(double), s));
      x_zero = true;
      break;
    case MBS_GUESS_DIAG:
      launch_axpby(c->ph.gamma, c->b.p, 0.0, c->xs.p, len, s);
      break;
    case MBS_GUESS_USER:
      if (!sigma0) return set_err(c, MBS_EINVAL, "MBS_GUESS_USER needs sigma0");
      launch_copy(sigma0, c->xs.p, len, s);
      break;
    case MBS_GUESS_LEARNED:
      CHK(learned_guess(c, n, R, p, c->b.p, c->xs.p, s));
      break;
    default:
      return set_err(c, MBS_EUNSUPPORTED, "guess %d not available", c->prm.guess);
  }
  double rel = 0.0;
  int rc = MBS_OK;
  OutPass op{v1s, v2s, v3t, Fz, Te, V, W, S};
  if (bnorm == 0.0) {
    HIPCHK(c, hipMemsetAsync(c->xs.p, 0, len * sizeof(double), s));
  } else if (c->prm.precision == MBS_FP64) {
    double res = 0.0;
    CHK(gmres(c, MBS_FP64, n, R, c->b.p, c->xs.p, x_zero, c->prm.tol * bnorm, c->prm.max_iter, true,
              &res, cnt, s, &op));
    rel = res / bnorm;
  } else {
    // mixed precision iterative refinement: binary64 residual rr = b - A64 x, binary32 inner
    // GMRES for the correction delta (zero start), x += delta, repeat.
    double* rr = c->dlt.p;
    CHK(ensure(c, c->stepbuf, len));
    double* delta = c->stepbuf.p;
    double beta;
    if (x_zero) {
      launch_copy(c->b.p, rr, len, s);
      beta = bnorm;
    } else {
      // The first residual only feeds the first inner solve, whose target (inner_tol) lies far above
      // the binary32 operator error, so it is formed with the binary32 operator; every later residual,
      // including the certified final one, is binary64.
      apply_op(c, MBS_FP32, n, R, c->xs.p, rr, s, cnt);
      launch_axpby(1.0, c->b.p, -1.0, rr, len, s);
      norm2(c, rr, len, sm.nsq, s);
      CHK(read_status(c, sm.nsq, 1, s));
      beta = sqrt(c->h_status[0]);
      if (beta <= c->prm.tol * bnorm) {
        // The guess may already pass (a configuration solved before): only a binary64 residual can
        // certify it, so form that one, with the outputs of the guess in the same pass.
        apply_op_out(c, n, R, c->xs.p, rr, op, s, cnt);
        launch_axpby(1.0, c->b.p, -1.0, rr, len, s);
        norm2(c, rr, len, sm.nsq, s);
        CHK(read_status(c, sm.nsq, 1, s));
        beta = sqrt(c->h_status[0]);
      }
    }
    while (beta > c->prm.tol * bnorm && cnt.iters < c->prm.max_iter) {
      HIPCHK(c, hipMemsetAsync(delta, 0, len * sizeof(double), s));
      // Inner target: inner_tol relative to the current residual, but no tighter than the final
      // tolerance needs (a fraction kLastStage of tol |b|), so the last stage stops as soon as the
      // binary64 residual can pass; the binary32 operator error (~1e-6 of |r|) stays far below it.
      constexpr double kLastStage = 0.3;
      const double target = std::max(c->prm.inner_tol * beta, kLastStage * c->prm.tol * bnorm);
      double inner = 0.0;
      CHK(gmres(c, MBS_FP32, n, R, rr, delta, true, target, c->prm.max_iter - cnt.iters, false, &inner,
                cnt, s));
      launch_axpby(1.0, delta, 1.0, c->xs.p, len, s);
      cnt.refinements++;
      if (target > c->prm.inner_tol * beta) {  // a last-stage target: expect this residual to pass
        apply_op_out(c, n, R, c->xs.p, rr, op, s, cnt);
      } else {
        apply_op(c, MBS_FP64, n, R, c->xs.p, rr, s, cnt);
        op.valid = false;
      }
      launch_axpby(1.0, c->b.p, -1.0, rr, len, s);
      norm2(c, rr, len, sm.nsq, s);
      CHK(read_status(c, sm.nsq, 1, s));
      beta = sqrt(c->h_status[0]);
    }
    rel = beta / bnorm;
  }
  if (bnorm != 0.0 && !(rel <= c->prm.tol)) rc = MBS_ENOCONV;
  HIPCHK(c, hipEventRecord(c->ev[2], s));
  const bool fused = op.valid;  // outputs already formed with the final residual
  if (!fused) {
    if (periodic(c))
      launch_per_out(R, v1s, v2s, v3t, Fz, Te, c->xs.p, V, W, S, c->part.p, n, per_box(c, n), c->ph, s);
    else
      launch_p3(R, v1s, v2s, v3t, Fz, Te, c->xs.p, V, W, S, c->part.p, n, c->ph, c->tile_pass, s);
    cnt.pairs += (double)n * (double)(n - 1);
    if (c->prm.plane) {
      launch_image_out(c->prm.plane, R, Fe, Te, c->xs.p, v3t, V, W, c->part.p, n, c->ph, c->prm.plane_z, s);
      cnt.pairs += (double)n * (double)n;
    }
  }
  if (high) {  // velocities and rotations from the septlet, vortlet and spinlet flows
    launch_high(1, R, n, R, n, hi, V, W, c->part.p, hsplit, c->ph, c->tile_pass, s);
    cnt.pairs += (double)n * (double)(n - 1);
  }
  if (Sigma) launch_copy(c->xs.p, Sigma, len, s);
  HIPCHK(c, hipEventRecord(c->ev[3], s));
  HIPCHK(c, hipStreamSynchronize(s));
  harvest_ops(c);
  if (st) {
    st->t_op64_ms = c->t_op[0];
    st->t_op32_ms = c->t_op[1];
    st->iters = cnt.iters;
    st->refinements = cnt.refinements;
    st->fp64_matvecs = cnt.f64;
    st->fp32_matvecs = cnt.f32;
    st->rel_resid = rel;
    st->t_rhs_ms = ev_ms(c->ev[0], c->ev[1]);
    st->t_iter_ms = ev_ms(c->ev[1], c->ev[2]);
    st->t_out_ms = fused ? ev_ms(c->ev[4], c->ev[5]) : ev_ms(c->ev[2], c->ev[3]);
    st->out_fused = fused ? 1 : 0;
    st->reserved = 0;
    st->t_total_ms = ev_ms(c->ev[0], c->ev[3]);
    st->pair_blocks = cnt.pairs;
  }
  if (rc == MBS_ENOCONV)
    set_err(c, MBS_ENOCONV, "no convergence: relative residual %.3e after %d iterations", rel,
            cnt.iters);
  return rc;
}

constexpr int64_t kSpatialOrderN = 65536;  // params.spatial_order = 0: reorder from this size on

// The solve without argument validation. With spatial ordering the inputs are gathered into the
// Morton order of the centres (the permutation of a cell grid with about two cells per sphere),
// solved in that order and the outputs scattered back, so that each workgroup's receivers are
// neighbours in space: binary32 coordinates relative to the first of them stay small and the
// neighbour lists' gathers stay local. The solution is the same up to the order of the sums.
int solve_core(mbs_ctx* c, int64_t n, const double* R, const double* p, const double* v1s, const double* v2s,
               const double* v3t, const double* Fe, const double* Te, const HighSlip& hi, const double* sigma0,
               double* V, double* W, double* S, double* Sigma, mbs_stats* st, hipStream_t s) {
  const int mode = c->prm.spatial_order;
  if (n < 2 || mode < 0 || (mode == 0 && n < kSpatialOrderN))
    return solve_in_order(c, n, R, p, v1s, v2s, v3t, Fe, Te, hi, sigma0, V, W, S, Sigma, st, s);
  const int64_t blk = (n + 63) / 64 * 64;  // doubles per row-width unit, padded
  CHK(ensure(c, c->ord, (size_t)blk * 71 + 64));
  double* base = c->ord.p;
  int32_t* perm = reinterpret_cast<int32_t*>(base);
  double* next = base + blk;  // the permutation takes n int32 <= blk doubles
  auto take = [&](int width) {
    double* q = next;
    next += (int64_t)width * blk;
    return q;
  };
  GridView g;
  CHK(grid_of(c, n, R, c->prm.a, 2 * n + 64, &g, s));
  HIPCHK(c, hipMemcpyAsync(perm, g.perm, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  auto gather = [&](const double* src, int width) -> const double* {
    if (!src) return nullptr;
    double* dst = take(width);
    launch_gather_rows(src, width, perm, n, dst, s);
    return dst;
  };
  const double* Ro = gather(R, 3);
  const double* po = gather(p, 3);
  const double* v1o = gather(v1s, 3);
  const double* v2o = gather(v2s, 5);
  const double* v3o = gather(v3t, 3);
  const double* Fo = gather(Fe, 3);
  const double* To = gather(Te, 3);
  const HighSlip hio{gather(hi.gam, 10), gather(hi.psi, 5), gather(hi.lam, 10)};
  const double* s0o = gather(c->prm.guess == MBS_GUESS_USER ? sigma0 : nullptr, 5);
  double* Vo = take(3);
  double* Wo = take(3);
  double* So = take(5);
  double* Sigo = Sigma ? take(5) : nullptr;
  HIPCHK(c, hipGetLastError());
  const int rc = solve_in_order(c, n, Ro, po, v1o, v2o, v3o, Fo, To, hio, s0o, Vo, Wo, So, Sigo, st, s);
  if (rc != MBS_OK && rc != MBS_ENOCONV) return rc;
  launch_scatter_rows(Vo, 3, perm, n, V, s);
  launch_scatter_rows(Wo, 3, perm, n, W, s);
  launch_scatter_rows(So, 5, perm, n, S, s);
  if (Sigma) launch_scatter_rows(Sigo, 5, perm, n, Sigma, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return rc;
}

// ---------------------------------------------------------------- static scratch (mbs_matvec_static)
// Device memory for callers that cannot allocate: the operator's chunk partial sums, packed source
// records and box centre of one application, for n <= kStaticMaxN. Every GPU the library runs on
// holds its own copy of this array until the process ends. Host code never uses the array's name
// as an address: its per-device address comes from hipGetSymbolAddress, taken once per device at
// context creation (with that device current) and kept in g_static_ptr.
constexpr int64_t kStaticMaxN = 131072;
constexpr size_t kStaticDoubles = (size_t)56 << 17;  // 56 MiB
__device__ __align__(256) double scratch[kStaticDoubles];

constexpr int kMaxDevices = 64;
double* g_static_ptr[kMaxDevices] = {};
std::mutex g_static_mu;

// Resolve this device's address of the scratch array (device current; once per device).
int attach_static_scratch(int device, std::string* msg) {
  if (device < 0 || device >= kMaxDevices) {
    *msg = "device index beyond the static scratch table";
    return MBS_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (g_static_ptr[device]) return MBS_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    *msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return MBS_EHIP;
  }
  g_static_ptr[device] = static_cast<double*>(ptr);
  return MBS_OK;
}

// Scratch of one operator application at launch shape t, in doubles, each region starting on a
// 256-byte boundary: chunk partial sums when the sources are split, packed source records for the
// scalar-streamed variant, the box centre.
struct OpScratch {
  int64_t part, src, orig, total;
};
OpScratch op_scratch(int64_t n, Tile t) {
  auto up = [](int64_t v) { return (v + 31) / 32 * 32; };
  const int tj = t.variant == 0 ? ((t.tj == 64 || t.tj == 256) ? t.tj : 128) : 64;
  const int split = split_for(n, t, tj);
  OpScratch o;
  o.part = 0;
  o.src = up(split > 1 ? (int64_t)split * 5 * n : 0);
  o.orig = o.src + up(t.variant == 1 ? 8 * n : 0);
  o.total = o.orig + 4;
  return o;
}

int begin_call(mbs_ctx* c) {
  if (!c) return MBS_EINVAL;
  c->err.clear();
  HIPCHK(c, hipSetDevice(c->device));
  return MBS_OK;
}

}  // namespace


// ---------------------------------------------------------------- traction ranks <= 3
// Unknowns x [n x 20] per sphere: [Sigma (5-basis), X^gam (7-basis), X^psi (5-basis), X^d (3)] (the
// flow stresslet and the equivalent slips of the septlet, vortlet and potential-dipole traction modes,
// section IV). The system is solved in binary64 by restarted GMRES without preconditioner; every
// operator application is one all-pairs pass of the rank-3 kernel.
namespace {

struct R3Ws {
  double *V, *w, *r, *b, *x, *zt, *na, *nb, *part;
};

int r3_workspace(mbs_ctx* c, int64_t n, R3Ws* o) {
  CHK(ensure_ws(c, n));  // dot partials, Hessenberg matrix, small vectors, zeros
  const int m = c->prm.restart;
  const int64_t len = 20 * n;
  const size_t total = (size_t)(m + 8) * len + (size_t)rank3_part_elems(n) + 64;
  CHK(ensure(c, c->r3, total));
  double* q = c->r3.p;
  o->V = q;
  q += (int64_t)(m + 1) * len;
  o->w = q;
  q += len;
  o->r = q;
  q += len;
  o->b = q;
  q += len;
  o->x = q;
  q += len;
  o->zt = q;
  q += len;
  o->na = q;
  q += len;
  o->nb = q;
  q += len;
  o->part = q;
  return MBS_OK;
}

// Right preconditioner of the rank <= 3 system: the near-field Neumann series of order k =
// params.near_order over the context's neighbour lists (near_prepare),
// y = sum_{i <= k} (-D^{-1} B_near)^i D^{-1} v, as t_1 = D^{-1}(v - B_near D^{-1} v),
// t_j = D^{-1}(v - B_near t_{j-1}), y = t_k (k passes; y must not overlap v)
void r3_precond(mbs_ctx* c, int64_t n, const double* R, const double* v, double* y, const R3Ws& ws,
                hipStream_t s) {
  const int* cntp = (const int*)c->near.p;
  const int order = near_order(c);
  if (order < 2) {
    launch_rank3_near(R, v, nullptr, cntp, cntp + n, n, c->ph, y, s);
    return;
  }
  double* ta = ws.na;
  double* tb = ws.nb;
  launch_rank3_near(R, v, nullptr, cntp, cntp + n, n, c->ph, ta, s);
  for (int j = 2; j < order; ++j) {
    launch_rank3_near(R, v, ta, cntp, cntp + n, n, c->ph, tb, s);
    double* t = ta;
    ta = tb;
    tb = t;
  }
  launch_rank3_near(R, v, ta, cntp, cntp + n, n, c->ph, y, s);
}

// y = A x (one pass), timed through the context's event ring like the rank-2 operator
void r3_apply(mbs_ctx* c, int64_t n, const double* R, const R3Ws& ws, const double* x, double* y, hipStream_t s,
              Counters& cnt) {
  if (c->npend == mbs_ctx::kRing) {
    (void)hipStreamSynchronize(s);
    harvest_ops(c);
  }
  const int slot = c->npend++;
  c->op_prec[slot] = MBS_FP64;
  (void)hipEventRecord(c->opev[2 * slot], s);
  launch_rank3(0, R, x, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, y, nullptr,
               nullptr, ws.part, n, c->ph, s);
  (void)hipEventRecord(c->opev[2 * slot + 1], s);
  cnt.f64++;
  cnt.pairs += (double)n * (double)(n - 1);
}

// Restarted GMRES(m) on the rank-3 system: classical Gram-Schmidt applied twice, Givens rotations on
// the device; with pc, right-preconditioned by r3_precond (A M^{-1} u = b, x = M^{-1} u); the
// residual of every restart is recomputed with the operator. *resid: final ||b - A x||.
int r3_gmres(mbs_ctx* c, int64_t n, const double* R, const R3Ws& ws, bool x_zero, bool pc, double tol_abs,
             int max_iters, double* resid, Counters& cnt, hipStream_t s) {
  const int m = c->prm.restart;
  const int64_t len = 20 * n;
  Small sm = small_of(c);
  if (x_zero) {
    launch_copy(ws.b, ws.r, len, s);
  } else {
    r3_apply(c, n, R, ws, ws.x, ws.r, s, cnt);
    launch_axpby(1.0, ws.b, -1.0, ws.r, len, s);
  }
  norm2(c, ws.r, len, sm.nsq, s);
  launch_init_g(sm.nsq, sm.g, m, sm.status, s);
  CHK(read_status(c, sm.status, 1, s));
  double beta = c->h_status[0];
  int used = 0;
  while (beta > tol_abs && used < max_iters) {
    launch_scale_by(ws.r, sm.status, 1, ws.V, len, s);
    int k = 0;
    bool breakdown = false;
    while (k < m && used < max_iters) {
      if (pc) {
        r3_precond(c, n, R, ws.V + (int64_t)k * len, ws.zt, ws, s);
        r3_apply(c, n, R, ws, ws.zt, ws.w, s, cnt);
      } else {
        r3_apply(c, n, R, ws, ws.V + (int64_t)k * len, ws.w, s, cnt);
      }
      launch_dots(ws.V, len, k + 1, ws.w, len, c->dpart.p, sm.h1, s);
      launch_axpy_multi(ws.V, len, k + 1, sm.h1, -1.0, ws.w, len, s);
      launch_dots(ws.V, len, k + 1, ws.w, len, c->dpart.p, sm.h2, s);
      launch_axpy_multi(ws.V, len, k + 1, sm.h2, -1.0, ws.w, len, s);
      norm2(c, ws.w, len, sm.nsq, s);
      launch_givens(c->H.p, m, k, sm.h1, sm.h2, sm.nsq, sm.cs, sm.sn, sm.g, sm.status, s);
      launch_scale_by(ws.w, sm.status + 1, 1, ws.V + (int64_t)(k + 1) * len, len, s);
      CHK(read_status(c, sm.status, 2, s));
      ++k;
      ++used;
      cnt.iters++;
      if (!(c->h_status[1] > 1e-300 * beta)) breakdown = true;
      if (c->h_status[0] <= tol_abs || breakdown) break;
    }
    launch_backsolve(c->H.p, m, k, sm.g, sm.y, s);
    if (pc) {  // x += M^{-1} (V y)
      launch_axpby(0.0, ws.w, 0.0, ws.zt, len, s);
      launch_axpy_multi(ws.V, len, k, sm.y, 1.0, ws.zt, len, s);
      r3_precond(c, n, R, ws.zt, ws.w, ws, s);
      launch_axpby(1.0, ws.w, 1.0, ws.x, len, s);
    } else {
      launch_axpy_multi(ws.V, len, k, sm.y, 1.0, ws.x, len, s);
    }
    r3_apply(c, n, R, ws, ws.x, ws.r, s, cnt);
    launch_axpby(1.0, ws.b, -1.0, ws.r, len, s);
    norm2(c, ws.r, len, sm.nsq, s);
    launch_init_g(sm.nsq, sm.g, m, sm.status, s);
    CHK(read_status(c, sm.status, 1, s));
    beta = c->h_status[0];
    if (breakdown) break;
  }
  *resid = beta;
  return MBS_OK;
}

int r3_check_n(mbs_ctx* c, int64_t n) {
  if (n < 1) return set_err(c, MBS_EINVAL, "n = %lld must be >= 1", (long long)n);
  if (n > (int64_t)INT32_MAX / 20) return set_err(c, MBS_EINVAL, "n too large");
  return MBS_OK;
}

}  // namespace

extern "C" {

void mbs_default_params(mbs_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->eta = 1.0 / (6.0 * M_PI);
  p->a = 1.0;
  p->tol = 1e-10;
  p->self_slip_c = 1.0;
  p->inner_tol = 1e-5;
  p->near_cutoff = 0.0;
  p->lmax = 2;
  p->max_iter = 300;
  p->restart = 30;
  p->precision = MBS_FP64;
  p->guess = MBS_GUESS_ZERO;
  p->check_overlap = 0;
  p->tile = 0;
  p->graph = 1;
  p->batch_item = 0;
  p->superposition = 0;
  p->near_order = 2;
  p->spatial_order = 0;
  p->plane = 0;
  p->plane_z = 0.0;
  p->box = 0.0;
  p->ewald_xi = 0.0;
  p->ewald_mesh = 0;
}

int mbs_create(mbs_ctx** out, int device, const mbs_params* prm) {
  g_create_error.clear();
  if (!out) return set_err(nullptr, MBS_EINVAL, "ctx pointer is NULL");
  *out = nullptr;
  mbs_params def;
  mbs_default_params(&def);
  if (!prm) prm = &def;
  int rc = validate_params(nullptr, prm);
  if (rc != MBS_OK) return rc;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return set_err(nullptr, MBS_EHIP, "hipGetDeviceCount: %s", hipGetErrorString(e));
  if (device < 0 || device >= ndev)
    return set_err(nullptr, MBS_EINVAL, "device %d out of range (%d devices)", device, ndev);
  e = hipSetDevice(device);
  if (e != hipSuccess) return set_err(nullptr, MBS_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
  {
    std::string msg;
    rc = attach_static_scratch(device, &msg);
    if (rc != MBS_OK) return set_err(nullptr, rc, "%s", msg.c_str());
  }
  mbs_ctx* c = new mbs_ctx();
  c->device = device;
  c->prm = *prm;
  c->ph = make_phys(prm->eta, prm->a, prm->self_slip_c);
  apply_tiles(c);
  e = hipHostMalloc((void**)&c->h_status, 8 * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void**)&c->d_count, 2 * sizeof(int));
  for (int k = 0; k < 8 && e == hipSuccess; ++k) e = hipEventCreate(&c->ev[k]);
  for (int k = 0; k < 2 * mbs_ctx::kRing && e == hipSuccess; ++k) e = hipEventCreate(&c->opev[k]);
  if (e != hipSuccess) {
    set_err(nullptr, MBS_EHIP, "context allocation: %s", hipGetErrorString(e));
    mbs_destroy(c);
    return MBS_EHIP;
  }
  *out = c;
  return MBS_OK;
}

void mbs_destroy(mbs_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  DevBuf* bufs[] = {&c->V, &c->w, &c->r, &c->b, &c->xs, &c->dlt, &c->part, &c->dpart,
                    &c->small, &c->H, &c->zeros, &c->stepbuf, &c->srcbuf, &c->orig, &c->near, &c->zt,
                    &c->nt, &c->stepstate,
                    &c->mlp_w, &c->mlp_g, &c->mlp_m, &c->mlp_v, &c->mlp_wb, &c->mlp_ws,
                    &c->mlp_part, &c->mlp_loss, &c->mlp_idx, &c->knn_buf, &c->grid, &c->ord, &c->r3, &c->per_kv, &c->per_seg, &c->per_tab, &c->per_mws, &c->per_rtab, &c->per_fws,
                    &c->bat, &c->btune};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (auto& g : c->bgraph)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto& sg : c->sgraph) sg.reset();
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  if (c->bstream) (void)hipStreamDestroy(c->bstream);
  if (c->d_count) (void)hipFree(c->d_count);
  if (c->h_status) (void)hipHostFree(c->h_status);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->opev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

int mbs_set_params(mbs_ctx* c, const mbs_params* prm) {
  CHK(begin_call(c));
  CHK(validate_params(c, prm));
  const bool restart_changed = prm->restart != c->prm.restart;
  c->prm = *prm;
  c->ph = make_phys(prm->eta, prm->a, prm->self_slip_c);
  apply_tiles(c);
  if (restart_changed) {  // buffers sized by restart are re-grown on demand
    DevBuf* bufs[] = {&c->V, &c->dpart, &c->small, &c->H};
    for (DevBuf* b : bufs) {
      if (b->p) (void)hipFree(b->p);
      b->p = nullptr;
      b->cap = 0;
    }
  }
  return MBS_OK;
}

const char* mbs_last_error(const mbs_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

namespace {
HighSlip high_of(const mbs_slip_ex* ex) {
  HighSlip h{nullptr, nullptr, nullptr};
  if (ex) {
    h.gam = ex->gam;
    h.psi = ex->psi;
    h.lam = ex->lam;
  }
  return h;
}
}  // namespace

int mbs_solve_ex(mbs_ctx* c, int64_t n, const double* R, const double* p, const double* v1s,
                 const double* v2s, const double* v3t, const mbs_slip_ex* ex, const double* Fe,
                 const double* Te, const double* sigma0, double* V, double* W, double* S, double* Sigma,
                 mbs_stats* st, void* stream) {
  CHK(begin_call(c));
  const HighSlip hi = high_of(ex);
  (void)p;
  if (n < 1) return set_err(c, MBS_EINVAL, "n = %lld must be >= 1", (long long)n);
  if (n > (int64_t)INT32_MAX / 6) return set_err(c, MBS_EINVAL, "n too large");
  if (!R || !V || !W || !S) return set_err(c, MBS_EINVAL, "R, V, W and S are required");
  if (c->prm.guess == MBS_GUESS_USER && !sigma0)
    return set_err(c, MBS_EINVAL, "MBS_GUESS_USER needs sigma0");
  if (c->prm.guess == MBS_GUESS_LEARNED) CHK(check_learned(c, n, p));
  const int64_t s0len = c->prm.guess == MBS_GUESS_USER ? 5 * n : 0;
  CHK(check_aliasing(c, {{"V", V, 3 * n}, {"W", W, 3 * n}, {"S", S, 5 * n}, {"Sigma", Sigma, 5 * n}},
                     {{"R", R, 3 * n}, {"p", p, 3 * n}, {"v1s", v1s, 3 * n}, {"v2s", v2s, 5 * n},
                      {"v3t", v3t, 3 * n}, {"Fe", Fe, 3 * n}, {"Te", Te, 3 * n}, {"sigma0", sigma0, s0len},
                      {"gam", hi.gam, 10 * n}, {"psi", hi.psi, 5 * n}, {"lam", hi.lam, 10 * n}}));
  hipStream_t s = (hipStream_t)stream;
  CHK(ensure_ws(c, n));
  CHK(check_inputs(c, s, {{R, 3 * n}, {v1s, 3 * n}, {v2s, 5 * n}, {v3t, 3 * n}, {Fe, 3 * n},
                          {Te, 3 * n}, {sigma0, s0len}, {hi.gam, 10 * n}, {hi.psi, 5 * n}, {hi.lam, 10 * n}},
                   p, n));
  if ((c->prm.plane || periodic(c)) && high_mask(hi))
    return set_err(c, MBS_EUNSUPPORTED, "the higher slip modes do not support params.plane or params.box");
  if (periodic(c) && c->prm.guess == MBS_GUESS_LEARNED)
    return set_err(c, MBS_EUNSUPPORTED, "the learned guess does not support params.box");
  CHK(check_plane(c, s, R, n));
  if (c->prm.check_overlap) {
    double md = 0.0;
    CHK(check_overlap(c, n, R, s, &md));
    if (md < 2.0 * c->prm.a)
      return set_err(c, MBS_EOVERLAP, "spheres overlap: minimum centre distance %.6g < 2a", md);
  }
  return solve_core(c, n, R, p, v1s, v2s, v3t, Fe, Te, hi, sigma0, V, W, S, Sigma, st, s);
}

int mbs_solve(mbs_ctx* c, int64_t n, const double* R, const double* p, const double* v1s,
              const double* v2s, const double* v3t, const double* Fe, const double* Te,
              const double* sigma0, double* V, double* W, double* S, double* Sigma, mbs_stats* st,
              void* stream) {
  return mbs_solve_ex(c, n, R, p, v1s, v2s, v3t, nullptr, Fe, Te, sigma0, V, W, S, Sigma, st, stream);
}


int mbs_matvec(mbs_ctx* c, int64_t n, const double* R, const double* x, double* y, int precision,
               void* stream) {
  CHK(begin_call(c));
  if (n < 1) return set_err(c, MBS_EINVAL, "n must be >= 1");
  if (n > (int64_t)INT32_MAX / 6) return set_err(c, MBS_EINVAL, "n too large");
  if (!R || !x || !y) return set_err(c, MBS_EINVAL, "R, x and y are required");
  CHK(check_aliasing(c, {{"y", y, 5 * n}}, {{"R", R, 3 * n}, {"x", x, 5 * n}}));
  if (precision != MBS_FP64 && precision != MBS_FP32)
    return set_err(c, MBS_EINVAL, "precision must be MBS_FP64 or MBS_FP32");
  hipStream_t s = (hipStream_t)stream;
  CHK(ensure_ws(c, n));
  CHK(check_plane(c, s, R, n));
  Counters cnt;
  c->npend = 0;
  apply_op(c, precision, n, R, x, y, s, cnt);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  c->npend = 0;
  return MBS_OK;
}

int mbs_matvec_static(mbs_ctx* c, int64_t n, const double* R, const double* x, double* y, int precision,
                      void* stream) {
  CHK(begin_call(c));
  CHK(refuse_plane(c, "mbs_matvec_static"));
  if (n < 1) return set_err(c, MBS_EINVAL, "n must be >= 1");
  if (n > kStaticMaxN)
    return set_err(c, MBS_EINVAL, "n = %lld exceeds the static scratch limit of %lld spheres", (long long)n,
                   (long long)kStaticMaxN);
  if (!R || !x || !y) return set_err(c, MBS_EINVAL, "R, x and y are required");
  CHK(check_aliasing(c, {{"y", y, 5 * n}}, {{"R", R, 3 * n}, {"x", x, 5 * n}}));
  if (precision != MBS_FP64 && precision != MBS_FP32)
    return set_err(c, MBS_EINVAL, "precision must be MBS_FP64 or MBS_FP32");
  double* base = g_static_ptr[c->device];
  if (!base) return set_err(c, MBS_EHIP, "static scratch not attached on device %d", c->device);
  const Tile t = precision == MBS_FP64 ? c->tile64 : c->tile32;
  const OpScratch sc = op_scratch(n, t);
  if (sc.total > (int64_t)kStaticDoubles)
    return set_err(c, MBS_EINVAL, "n = %lld needs %lld doubles of scratch at this launch shape (static scratch: %zu)",
                   (long long)n, (long long)sc.total, kStaticDoubles);
  // every region is written before it is read within the application, so nothing needs clearing
  double* src = base + sc.src;
  double* orig = base + sc.orig;
  hipStream_t s = (hipStream_t)stream;
  launch_p2(precision == MBS_FP32, R, x, y, base, src, orig, n, c->ph, t, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_rhs_ex(mbs_ctx* c, int64_t n, const double* R, const double* v2s, const double* v3t,
               const mbs_slip_ex* ex, const double* Fe, const double* Te, double* b, void* stream) {
  CHK(begin_call(c));
  if (n < 1) return set_err(c, MBS_EINVAL, "n must be >= 1");
  if (n > (int64_t)INT32_MAX / 10) return set_err(c, MBS_EINVAL, "n too large");
  if (!R || !b) return set_err(c, MBS_EINVAL, "R and b are required");
  const HighSlip hi = high_of(ex);
  CHK(check_aliasing(c, {{"b", b, 5 * n}},
                     {{"R", R, 3 * n}, {"v2s", v2s, 5 * n}, {"v3t", v3t, 3 * n}, {"Fe", Fe, 3 * n},
                      {"Te", Te, 3 * n}, {"gam", hi.gam, 10 * n}, {"psi", hi.psi, 5 * n}, {"lam", hi.lam, 10 * n}}));
  hipStream_t s = (hipStream_t)stream;
  CHK(ensure_ws(c, n));
  if ((c->prm.plane || periodic(c)) && high_mask(hi))
    return set_err(c, MBS_EUNSUPPORTED, "the higher slip modes do not support params.plane or params.box");
  CHK(check_plane(c, s, R, n));
  if (periodic(c))
    launch_per_rhs(R, v2s, v3t, Fe ? Fe : c->zeros.p, Te, b, c->part.p, n, per_box(c, n), c->ph, s);
  else
    launch_p1(R, v2s, v3t, Fe ? Fe : c->zeros.p, Te, b, c->part.p, n, c->ph, c->tile_pass, s);
  if (high_mask(hi))
    launch_high(0, R, n, R, n, hi, b, nullptr, c->part.p, high_split(n, n, c->tile_pass), c->ph, c->tile_pass, s);
  if (c->prm.plane) launch_image_rhs(c->prm.plane, R, Fe, Te, v3t, b, c->part.p, n, c->ph, c->prm.plane_z, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_rhs(mbs_ctx* c, int64_t n, const double* R, const double* v2s, const double* v3t,
            const double* Fe, const double* Te, double* b, void* stream) {
  return mbs_rhs_ex(c, n, R, v2s, v3t, nullptr, Fe, Te, b, stream);
}

int mbs_outputs_ex(mbs_ctx* c, int64_t n, const double* R, const double* v1s, const double* v2s,
                   const double* v3t, const mbs_slip_ex* ex, const double* Fe, const double* Te,
                   const double* Sigma, double* V, double* W, double* S, void* stream) {
  CHK(begin_call(c));
  if (n < 1) return set_err(c, MBS_EINVAL, "n must be >= 1");
  if (n > (int64_t)INT32_MAX / 10) return set_err(c, MBS_EINVAL, "n too large");
  if (!R || !Sigma || !V || !W) return set_err(c, MBS_EINVAL, "R, Sigma, V and W are required");
  const HighSlip hi = high_of(ex);
  CHK(check_aliasing(c, {{"V", V, 3 * n}, {"W", W, 3 * n}, {"S", S, 5 * n}},
                     {{"R", R, 3 * n}, {"v1s", v1s, 3 * n}, {"v2s", v2s, 5 * n}, {"v3t", v3t, 3 * n},
                      {"Fe", Fe, 3 * n}, {"Te", Te, 3 * n}, {"Sigma", Sigma, 5 * n}, {"gam", hi.gam, 10 * n},
                      {"psi", hi.psi, 5 * n}, {"lam", hi.lam, 10 * n}}));
  hipStream_t s = (hipStream_t)stream;
  CHK(ensure_ws(c, n));
  if ((c->prm.plane || periodic(c)) && high_mask(hi))
    return set_err(c, MBS_EUNSUPPORTED, "the higher slip modes do not support params.plane or params.box");
  CHK(check_plane(c, s, R, n));
  if (periodic(c))
    launch_per_out(R, v1s, v2s, v3t, Fe ? Fe : c->zeros.p, Te, Sigma, V, W, S, c->part.p, n, per_box(c, n), c->ph, s);
  else
    launch_p3(R, v1s, v2s, v3t, Fe ? Fe : c->zeros.p, Te, Sigma, V, W, S, c->part.p, n, c->ph, c->tile_pass, s);
  if (high_mask(hi))
    launch_high(1, R, n, R, n, hi, V, W, c->part.p, high_split(n, n, c->tile_pass), c->ph, c->tile_pass, s);
  if (c->prm.plane)
    launch_image_out(c->prm.plane, R, Fe, Te, Sigma, v3t, V, W, c->part.p, n, c->ph, c->prm.plane_z, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_outputs(mbs_ctx* c, int64_t n, const double* R, const double* v1s, const double* v2s,
                const double* v3t, const double* Fe, const double* Te, const double* Sigma,
                double* V, double* W, double* S, void* stream) {
  return mbs_outputs_ex(c, n, R, v1s, v2s, v3t, nullptr, Fe, Te, Sigma, V, W, S, stream);
}

int mbs_flow_ex(mbs_ctx* c, int64_t m, const double* X, int64_t n, const double* R, const double* Fe,
                const double* Te, const double* Sigma, const double* v3t, const mbs_slip_ex* ex, double* U,
                void* stream) {
  CHK(begin_call(c));
  if (m < 1 || n < 1) return set_err(c, MBS_EINVAL, "m and n must be >= 1");
  if (m > (int64_t)INT32_MAX / 12 || n > (int64_t)INT32_MAX / 10) return set_err(c, MBS_EINVAL, "m or n too large");
  if (!X || !R || !Sigma || !U) return set_err(c, MBS_EINVAL, "X, R, Sigma and U are required");
  const HighSlip hi = high_of(ex);
  CHK(check_aliasing(c, {{"U", U, 3 * m}},
                     {{"X", X, 3 * m}, {"R", R, 3 * n}, {"Fe", Fe, 3 * n}, {"Te", Te, 3 * n},
                      {"Sigma", Sigma, 5 * n}, {"v3t", v3t, 3 * n}, {"gam", hi.gam, 10 * n},
                      {"psi", hi.psi, 5 * n}, {"lam", hi.lam, 10 * n}}));
  hipStream_t s = (hipStream_t)stream;
  CHK(ensure_ws(c, n));  // (zeros stand in for absent forces)
  if (periodic(c)) {  // the periodic suspension's flow (Ewald sums)
    if (high_mask(hi)) return set_err(c, MBS_EUNSUPPORTED, "the higher slip modes do not support params.box");
    CHK(ensure(c, c->part, (size_t)per_part_elems(m, n, c->per_K, c->per_nseg8)));
    PerBox g = per_box(c, n);
    if (g.M > 0 && g.nc >= 3) {  // the field points binned like the spheres: real space over cells
      g.fws_bytes = pm_flow_ws_bytes(m, g.nc);
      CHK(ensure(c, c->per_fws, (g.fws_bytes + 7) / 8));
      g.fws = c->per_fws.p;
    }
    launch_per_flow(X, m, R, n, Fe, Te, Sigma, v3t, U, c->part.p, g, c->ph, s);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(s));
    return MBS_OK;
  }
  const int hsplit = high_split(m, n, c->tile_pass);
  CHK(ensure(c, c->part, (size_t)std::max<int64_t>((int64_t)std::max(flow_split(m, n, c->tile_pass), high_mask(hi) ? hsplit : 0) * 3 * m,
                                                 c->prm.plane ? image_part_elems(m, n) : 0) + 64));
  if (c->prm.plane) {
    if (high_mask(hi))
      return set_err(c, MBS_EUNSUPPORTED, "the higher slip modes do not support params.plane");
    CHK(check_plane(c, s, R, n));
    CHK(check_above(c, s, X, m, c->prm.plane_z, "field points lie below the plane"));
  }
  launch_flow(X, m, R, Fe ? Fe : c->zeros.p, Te, Sigma, v3t, U, c->part.p, n, c->ph, c->tile_pass, s);
  if (high_mask(hi)) launch_high(2, X, m, R, n, hi, U, nullptr, c->part.p, hsplit, c->ph, c->tile_pass, s);
  if (c->prm.plane)
    launch_image_flow(c->prm.plane, X, m, R, n, Fe, Te, Sigma, v3t, U, c->part.p, c->ph, c->prm.plane_z, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_flow(mbs_ctx* c, int64_t m, const double* X, int64_t n, const double* R, const double* Fe,
             const double* Te, const double* Sigma, const double* v3t, double* U, void* stream) {
  return mbs_flow_ex(c, m, X, n, R, Fe, Te, Sigma, v3t, nullptr, U, stream);
}

int mbs_step(mbs_ctx* c, int64_t n, double* R, double* p, double k_trap, const double* slip_coef,
             double dt, int32_t nsteps, int32_t order, double* hist, int32_t hist_valid,
             mbs_stats* per_step, double* min_dist, void* stream) {
  CHK(begin_call(c));
  if (n < 1) return set_err(c, MBS_EINVAL, "n must be >= 1");
  if (n > (int64_t)INT32_MAX / 6) return set_err(c, MBS_EINVAL, "n too large");
  if (!R || !p || !slip_coef) return set_err(c, MBS_EINVAL, "R, p and slip_coef are required");
  if (nsteps < 0) return set_err(c, MBS_EINVAL, "nsteps must be >= 0");
  if (order != 1 && order != 2) return set_err(c, MBS_EINVAL, "order must be 1 or 2");
  if (!isfinite(dt) || !isfinite(k_trap)) return set_err(c, MBS_EINVAL, "dt and k must be finite");
  if (hist_valid && !hist) return set_err(c, MBS_EINVAL, "hist_valid needs hist");
  if (c->prm.guess == MBS_GUESS_LEARNED) CHK(check_learned(c, n, p));
  CHK(check_aliasing(c, {{"R", R, 3 * n}, {"p", p, 3 * n}, {"hist", hist, 11 * n}}, {}));
  hipStream_t s = (hipStream_t)stream;
  CHK(ensure_ws(c, n));
  // state: Fe, v1s, v3t, V, W, Vprev, Pdprev [3n] each; v2s, Sigma, S [5n] each. Vprev, Pdprev and
  // Sigma are the history that hist carries in and out (in that order, 11n values).
  const size_t need = (size_t)(3 * 7 + 5 * 3) * n;
  CHK(ensure(c, c->stepstate, need));
  double* Fe = c->stepstate.p;
  double* v1s = Fe + 3 * n;
  double* v3t = v1s + 3 * n;
  double* V = v3t + 3 * n;
  double* W = V + 3 * n;
  double* Vp = W + 3 * n;
  double* Pp = Vp + 3 * n;
  double* v2s = Pp + 3 * n;
  double* Sg = v2s + 5 * n;
  double* Sout = Sg + 5 * n;
  int rc = check_inputs(c, s, {{R, 3 * n}, {hist_valid ? hist : nullptr, 11 * n}}, p, n);
  if (rc == MBS_OK) rc = check_plane(c, s, R, n);
  const int guess0 = c->prm.guess;
  bool noconv = false;
  if (rc == MBS_OK && hist_valid) {  // resume: the previous step's V, Omega x p and Sigma
    launch_copy(hist, Vp, 3 * n, s);
    launch_copy(hist + 3 * n, Pp, 3 * n, s);
    launch_copy(hist + 6 * n, Sg, 5 * n, s);
  }
  for (int k = 0; k < nsteps && rc == MBS_OK; ++k) {
    launch_trap_modes(R, p, k_trap, slip_coef[0], slip_coef[1], slip_coef[2], Fe, v1s, v2s, v3t, n,
                      s);
    // above a plane the run goes on while every centre is above it (closer than a is contact with
    // it, as a pair closer than 2a is, and the model has no steric force); each sphere's own image
    // counts as a neighbour at distance 2h in min_dist
    double hmin = INFINITY;
    if (c->prm.plane) {
      rc = min_height(c, n, R, s, &hmin);
      if (rc != MBS_OK) break;
      if (!(hmin > 0.0)) {
        rc = set_err(c, MBS_EINVAL, "step %d: a sphere centre reached the plane", k);
        break;
      }
    }
    if (min_dist) {
      double md = 0.0;
      rc = periodic(c) ? per_min_dist(c, n, R, s, &md) : check_overlap(c, n, R, s, &md);
      if (rc != MBS_OK) break;
      min_dist[k] = fmin(md, 2.0 * hmin);
    }
    mbs_stats one{};
    const bool first = k == 0 && !hist_valid;  // no history yet: one-body guess, Euler step
    const bool warm = guess0 == MBS_GUESS_USER && !first;
    if (guess0 == MBS_GUESS_USER && first) c->prm.guess = MBS_GUESS_DIAG;
    rc = solve_core(c, n, R, p, v1s, v2s, slip_coef[2] != 0.0 ? v3t : nullptr, Fe, nullptr, HighSlip{nullptr, nullptr, nullptr},
                    warm ? Sg : nullptr, V, W, Sout, Sg, &one, s);
    c->prm.guess = guess0;
    if (rc != MBS_OK && rc != MBS_ENOCONV) break;
    if (per_step) per_step[k] = one;
    // a step whose solve stopped short of the tolerance still advances (it is reported through
    // per_step[k].rel_resid); a non-finite residual ends the run
    if (!isfinite(one.rel_resid)) break;
    launch_ab_update(R, p, V, W, Vp, Pp, dt, first, order, n, s);
    if (rc == MBS_ENOCONV) {
      noconv = true;
      rc = MBS_OK;
    }
  }
  if (rc == MBS_OK && noconv) {
    rc = MBS_ENOCONV;
    set_err(c, MBS_ENOCONV, "some steps stopped short of the tolerance (see per-step rel_resid)");
  }
  if (hist && (rc == MBS_OK || rc == MBS_ENOCONV) && (nsteps > 0 || hist_valid)) {
    launch_copy(Vp, hist, 3 * n, s);
    launch_copy(Pp, hist + 3 * n, 3 * n, s);
    launch_copy(Sg, hist + 6 * n, 5 * n, s);
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess && rc == MBS_OK) rc = set_err(c, MBS_EHIP, "%s", hipGetErrorString(e));
  return rc;
}

namespace {

// Work items (configuration, first receiver) of `item` receivers each, largest configurations
// first: an item's work is its configuration's size, and workgroups start in index order, so the
// long items start early and the short ones fill the tail of each pass.
void batch_items(const std::vector<int>& off, int nconf, int item, std::vector<int2>& items) {
  items.clear();
  for (int b = 0; b < nconf; ++b)
    for (int r = off[b]; r < off[b + 1]; r += item) items.push_back(make_int2(b, r));
  std::stable_sort(items.begin(), items.end(), [&](const int2& u, const int2& v) {
    return off[u.x + 1] - off[u.x] > off[v.x + 1] - off[v.x];
  });
}

int check_offsets(mbs_ctx* c, int32_t nconf, const int64_t* offsets) {
  if (nconf < 1 || !offsets) return set_err(c, MBS_EINVAL, "nconf >= 1 and offsets are required");
  if (offsets[0] != 0) return set_err(c, MBS_EINVAL, "offsets[0] must be 0");
  for (int b = 0; b < nconf; ++b)
    if (offsets[b + 1] <= offsets[b]) return set_err(c, MBS_EINVAL, "offsets must increase");
  if (offsets[nconf] > (int64_t)INT32_MAX / 20) return set_err(c, MBS_EINVAL, "too many spheres in the batch");
  return MBS_OK;
}

}  // namespace

int mbs_solve_batched(mbs_ctx* c, int32_t nconf, const int64_t* offsets, const double* R,
                      const double* v1s, const double* v2s, const double* v3t, const double* Fe,
                      const double* Te, double* V, double* W, double* S, double* Sigma,
                      mbs_stats* per_conf, double* latency_ms, void* stream) {
  CHK(begin_call(c));
  CHK(refuse_plane(c, "mbs_solve_batched"));
  CHK(check_offsets(c, nconf, offsets));
  if (!R || !V || !W || !S) return set_err(c, MBS_EINVAL, "R, V, W and S are required");
  const int64_t ntot64 = offsets[nconf];
  const int ntot = (int)ntot64;
  CHK(check_aliasing(c, {{"V", V, 3 * ntot64}, {"W", W, 3 * ntot64}, {"S", S, 5 * ntot64}, {"Sigma", Sigma, 5 * ntot64}},
                     {{"R", R, 3 * ntot64}, {"v1s", v1s, 3 * ntot64}, {"v2s", v2s, 5 * ntot64},
                      {"v3t", v3t, 3 * ntot64}, {"Fe", Fe, 3 * ntot64}, {"Te", Te, 3 * ntot64}}));
  hipStream_t s = (hipStream_t)stream;
  int bad = 0;
  CHK(ensure_ws(c, 16));
  CHK(count_nonfinite(c, s, {{R, 3 * ntot64}, {v1s, 3 * ntot64}, {v2s, 5 * ntot64}, {v3t, 3 * ntot64},
                             {Fe, 3 * ntot64}, {Te, 3 * ntot64}},
                      &bad));
  if (bad) return set_err(c, MBS_EINVAL, "%d non-finite input values", bad);
  if (c->prm.precision != MBS_FP64)
    return set_err(c, MBS_EUNSUPPORTED, "batched solves run in binary64 only");
  // host descriptors: configuration offsets, work items (configuration, receiver tile), owner map;
  // built and uploaded unless the previous batch had the same offsets, item size and workspace
  const int m = c->prm.restart;
  std::vector<int> off, cid;
  std::vector<int2> items;
  const int item = c->prm.batch_item ? c->prm.batch_item : c->bitem;
  const bool same_desc = c->bdesc_item == item && (int64_t)c->bdesc_off.size() == (int64_t)nconf + 1 &&
                         std::equal(c->bdesc_off.begin(), c->bdesc_off.end(), offsets);
  if (!same_desc) {
    off.resize(nconf + 1);
    cid.resize(ntot);
    for (int b = 0; b <= nconf; ++b) off[b] = (int)offsets[b];
    for (int b = 0; b < nconf; ++b)
      for (int r = off[b]; r < off[b + 1]; ++r) cid[r] = b;
    batch_items(off, nconf, item, items);
  }
  const int nitems = same_desc ? c->bdesc_nitems : (int)items.size();
  // workspace (bytes, 256-aligned pieces)
  const int64_t len = 5 * ntot64;
  const int hs = m + 2;
  size_t bytes = 0;
  auto reserve = [&](size_t b) { size_t o = bytes; bytes += align256(b); return o; };
  const int C = 4;  // Arnoldi steps per round
  // Krylov basis: m + 1 vectors and C spare ones, so that the preconditioner of the steps left in a
  // round after every cycle has ended reads inside the basis (their results are not used)
  const size_t oV = reserve((size_t)(m + 1 + C) * len * 8), ow = reserve(len * 8), ox = reserve(len * 8),
               ob = reserve(len * 8), orr = reserve(len * 8), orec = reserve((size_t)ntot * sizeof(RecO)),
               oH = reserve((size_t)nconf * (m + 1) * (m + 1) * 8);
  size_t osm[7];
  for (int k = 0; k < 7; ++k) osm[k] = reserve((size_t)nconf * hs * 8);  // cs sn g y h1 h2 spare
  const size_t onsq = reserve(nconf * 8), obn = reserve(nconf * 8), ohk = reserve(nconf * 8),
               ores = reserve(nconf * 8), ost = reserve(nconf * 4), oke = reserve(nconf * 4),
               oit = reserve(nconf * 4), ot0 = reserve(nconf * 8), ot1 = reserve(nconf * 8),
               okd = reserve(16), ocnt = reserve(16), ooff = reserve((nconf + 1) * 4),
               oitems = reserve((size_t)nitems * 8), ocid = reserve((size_t)ntot * 4);
  // near-field preconditioner: lists (counts, then kNearCap entries per sphere) and three vectors
  const bool pc = c->prm.near_cutoff > 0.0;
  const size_t onear = pc ? reserve((size_t)ntot * (kNearCap + 1) * 4) : 0,
               ozt = pc ? reserve(len * 8) : 0, out_ = pc ? reserve(len * 8) : 0,
               ont = pc ? reserve(2 * len * 8) : 0;
  const void* bat0 = c->bat.p;
  const size_t batcap0 = c->bat.cap;
  CHK(ensure(c, c->bat, bytes / 8 + 64));
  if (c->bat.p != bat0 || c->bat.cap != batcap0) c->bdesc_off.clear();  // reallocated: contents gone
  char* base = (char*)c->bat.p;
  double* Vb = (double*)(base + oV);
  double *wv = (double*)(base + ow), *xv = (double*)(base + ox), *bv = (double*)(base + ob),
         *rv = (double*)(base + orr);
  void* rec = base + orec;
  BatchState st;
  st.H = (double*)(base + oH);
  st.cs = (double*)(base + osm[0]);
  st.sn = (double*)(base + osm[1]);
  st.g = (double*)(base + osm[2]);
  st.y = (double*)(base + osm[3]);
  st.h1 = (double*)(base + osm[4]);
  st.h2 = (double*)(base + osm[5]);
  st.nsq = (double*)(base + onsq);
  st.bnorm = (double*)(base + obn);
  st.hk1 = (double*)(base + ohk);
  st.resid = (double*)(base + ores);
  st.status = (int*)(base + ost);
  st.kend = (int*)(base + oke);
  st.iters = (int*)(base + oit);
  st.t0 = (unsigned long long*)(base + ot0);
  st.t1 = (unsigned long long*)(base + ot1);
  int* kdev = (int*)(base + okd);
  int* dcnt = (int*)(base + ocnt);
  int* doff = (int*)(base + ooff);
  int2* ditems = (int2*)(base + oitems);
  int* dcid = (int*)(base + ocid);
  int* ncnt = pc ? (int*)(base + onear) : nullptr;
  int* nlist = pc ? ncnt + ntot : nullptr;
  double* zt = pc ? (double*)(base + ozt) : nullptr;
  double* nt = pc ? (double*)(base + ont) : nullptr;
  double* ut = pc ? (double*)(base + out_) : nullptr;
  const double near_rc = c->prm.near_cutoff, near_rmin = 2.0 * c->prm.a;
  if (!same_desc || c->bdesc_off.empty() || c->bdesc_ptr[0] != (void*)doff || c->bdesc_ptr[1] != (void*)ditems ||
      c->bdesc_ptr[2] != (void*)dcid) {
    if (same_desc) {  // same batch, moved or lost device copies: rebuild the host copies first
      off.resize(nconf + 1);
      cid.resize(ntot);
      for (int b = 0; b <= nconf; ++b) off[b] = (int)offsets[b];
      for (int b = 0; b < nconf; ++b)
        for (int r = off[b]; r < off[b + 1]; ++r) cid[r] = b;
      batch_items(off, nconf, item, items);
    }
    c->bdesc_off.clear();  // invalid until the uploads below have completed
    HIPCHK(c, hipMemcpyAsync(doff, off.data(), (nconf + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(ditems, items.data(), nitems * sizeof(int2), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(dcid, cid.data(), ntot * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));  // the host vectors go out of scope with this call
    if (!same_desc) ++c->bdesc_gen;
    c->bdesc_off.assign(offsets, offsets + nconf + 1);
    c->bdesc_item = item;
    c->bdesc_nitems = nitems;
    c->bdesc_ptr[0] = doff;
    c->bdesc_ptr[1] = ditems;
    c->bdesc_ptr[2] = dcid;
  }
  if (!c->bstream) HIPCHK(c, hipStreamCreateWithFlags(&c->bstream, hipStreamNonBlocking));
  hipStream_t bs = c->bstream;
  // the batch stream waits for the caller's stream (uploads above, caller's producers)
  HIPCHK(c, hipEventRecord(c->ev[4], s));
  HIPCHK(c, hipStreamWaitEvent(bs, c->ev[4], 0));
  const Phys ph = c->ph;
  const double tol = c->prm.tol;
  const int max_iter = c->prm.max_iter;
  const bool has_t = Te != nullptr, has_d = v3t != nullptr;
  // the four phases
  auto phase_init = [&](hipStream_t q) {
    batched_set_ints(st.status, nconf, kActive, q);
    batched_pack_f(R, Fe, Te, v3t, ph, (RecF*)rec, ntot, q);
    batched_p1(ditems, nitems, item, doff, (const RecF*)rec, v2s, has_t, has_d, ph, bv, q);
    if (pc) batched_near_build(ditems, nitems, item, doff, R, near_rmin, near_rc, ncnt, nlist, q);
    batched_fill(xv, 0.0, len, q);
    batched_dots(bv, 0, nullptr, 1, bv, doff, st.status, kActive, st.nsq, 1, nconf, q);
    batched_init(st, nconf, m, q);
    batched_start(bv, st.hk1, dcid, st.status, kActive, Vb, len, q);
    batched_set_int(kdev, 0, q);
  };
  // One round: C Arnoldi steps of every active configuration, then the certification of every
  // configuration whose cycle ended (iterate update, true residual: final, or waiting to restart),
  // the restart gate, and the count of configurations not yet final.
  auto phase_round = [&](hipStream_t q) {
    for (int it = 0; it < C; ++it) {
      if (pc) {  // right preconditioning: w = A M^{-1} v_k
        launch_near_apply(R, Vb, ncnt, nlist, ntot, ph, zt, q, kdev, len, nt, near_order(c));
        batched_pack_s(R, zt, nullptr, 0, 0, (Src8<double>*)rec, ntot, q);
        batched_p2(ditems, nitems, item, doff, st.status, kActive, (const Src8<double>*)rec, zt, nullptr, 0, ph, wv,
                   q);
      } else {
        batched_pack_s(R, Vb, kdev, m - 1, len, (Src8<double>*)rec, ntot, q);
        batched_p2(ditems, nitems, item, doff, st.status, kActive, (const Src8<double>*)rec, Vb, kdev, len, ph, wv,
                   q);
      }
      batched_dots(Vb, len, kdev, 0, wv, doff, st.status, kActive, st.h1, hs, nconf, q);
      batched_axpy(Vb, len, kdev, nullptr, 0, st.h1, hs, -1.0, dcid, st.status, kActive, wv, len, q);
      batched_dots(Vb, len, kdev, 0, wv, doff, st.status, kActive, st.h2, hs, nconf, q);
      batched_axpy(Vb, len, kdev, nullptr, 0, st.h2, hs, -1.0, dcid, st.status, kActive, wv, len, q);
      batched_dots(wv, 0, nullptr, 1, wv, doff, st.status, kActive, st.nsq, 1, nconf, q);
      batched_givens(st, nconf, m, kdev, tol, max_iter, q);
      batched_scale(wv, st.hk1, dcid, st.status, Vb, len, kdev, len, q);
      batched_inc(kdev, q);
    }
    batched_backsolve(st, nconf, m, q);
    if (pc) {  // x += M^{-1} (V y) for the configurations that ended a cycle (zero elsewhere)
      batched_fill(ut, 0.0, len, q);
      batched_axpy(Vb, len, nullptr, st.kend, 0, st.y, hs, 1.0, dcid, st.status, kCycleDone, ut, len, q);
      launch_near_apply(R, ut, ncnt, nlist, ntot, ph, zt, q, nullptr, 0, nt, near_order(c));
      launch_axpby(1.0, zt, 1.0, xv, len, q);
    } else {
      batched_axpy(Vb, len, nullptr, st.kend, 0, st.y, hs, 1.0, dcid, st.status, kCycleDone, xv, len, q);
    }
    batched_pack_s(R, xv, nullptr, 0, 0, (Src8<double>*)rec, ntot, q);
    batched_p2(ditems, nitems, item, doff, st.status, kCycleDone, (const Src8<double>*)rec, xv, nullptr, 0, ph,
               wv, q);
    batched_resid(bv, wv, dcid, st.status, rv, len, q);
    batched_dots(rv, 0, nullptr, 1, rv, doff, st.status, kCycleDone, st.nsq, 1, nconf, q);
    batched_check(st, nconf, m, tol, max_iter, q);
    batched_start(rv, st.hk1, dcid, st.status, kRestart, Vb, len, q);
    batched_gate(st.status, nconf, kdev, q);
    batched_count_not(st.status, nconf, kFinal, dcnt, q);
  };
  auto phase_out = [&](hipStream_t q) {
    batched_pack_o(R, Fe, Te, xv, v3t, ph, (RecO*)rec, ntot, q);
    batched_p3(ditems, nitems, item, doff, (const RecO*)rec, has_t, has_d, ph, v1s, v2s, Fe, Te, xv, V, W, S,
               Sigma, q);
  };
  // graphs: captured once per batch shape (pointers and sizes), replayed afterwards
  const bool use_graph = c->prm.graph != 0;
  auto capture = [&](hipGraphExec_t* exec, const std::function<void(hipStream_t)>& body) -> int {
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(bs, hipStreamCaptureModeThreadLocal));
    body(bs);
    HIPCHK(c, hipStreamEndCapture(bs, &g));
    hipError_t e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      *exec = nullptr;
      return set_err(c, MBS_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return MBS_OK;
  };
  if (use_graph) {
    std::vector<uintptr_t> key = {(uintptr_t)nconf, (uintptr_t)ntot, (uintptr_t)base, (uintptr_t)R,
                                  (uintptr_t)v1s, (uintptr_t)v2s, (uintptr_t)v3t, (uintptr_t)Fe,
                                  (uintptr_t)Te, (uintptr_t)V, (uintptr_t)W, (uintptr_t)S,
                                  (uintptr_t)Sigma, (uintptr_t)m, (uintptr_t)max_iter};
    double tolc = tol;
    uintptr_t tb;
    memcpy(&tb, &tolc, sizeof tb);
    key.push_back(tb);
    double cs_ = ph.c_slip, eta_ = ph.eta, a_ = ph.a, rc_ = near_rc;
    memcpy(&tb, &cs_, sizeof tb);
    key.push_back(tb);
    memcpy(&tb, &rc_, sizeof tb);
    key.push_back(tb);
    key.push_back((uintptr_t)item);
    key.push_back((uintptr_t)nitems);
    key.push_back((uintptr_t)c->bdesc_gen);  // the captured launches depend on the batch's items
    key.push_back((uintptr_t)near_order(c));
    memcpy(&tb, &eta_, sizeof tb);
    key.push_back(tb);
    memcpy(&tb, &a_, sizeof tb);
    key.push_back(tb);
    if (key != c->bkey || !c->bgraph[0]) {
      for (auto& g : c->bgraph)
        if (g) {
          (void)hipGraphExecDestroy(g);
          g = nullptr;
        }
      c->bkey.clear();
      c->bwhole_rounds = 0;
      CHK(capture(&c->bgraph[0], phase_init));
      CHK(capture(&c->bgraph[1], phase_round));
      CHK(capture(&c->bgraph[2], phase_out));
      c->bkey = key;
    }
  }
  auto run = [&](int k) -> int {
    if (use_graph) {
      HIPCHK(c, hipGraphLaunch(c->bgraph[k], bs));
    } else {
      if (k == 0) phase_init(bs);
      if (k == 1) phase_round(bs);
      if (k == 2) phase_out(bs);
      HIPCHK(c, hipGetLastError());
    }
    return MBS_OK;
  };
  auto remaining = [&](int* out) -> int {  // configurations not yet final
    HIPCHK(c, hipMemcpyAsync(out, dcnt, sizeof(int), hipMemcpyDeviceToHost, bs));
    HIPCHK(c, hipStreamSynchronize(bs));
    return MBS_OK;
  };
  const int max_rounds = max_iter / C + 2 * (max_iter / std::max(1, m) + 2);
  HIPCHK(c, hipEventRecord(c->ev[5], bs));
  int left = 1, whole_rounds = 0;
  if (use_graph && c->bgraph[3]) {
    // the whole solve in one launch, sized by the rounds the last solve of this shape took; the host
    // reads one counter at the end and continues round by round only if some configuration is left
    HIPCHK(c, hipGraphLaunch(c->bgraph[3], bs));
    CHK(remaining(&left));
    if (left > 0) {
      int rounds = c->bwhole_rounds;
      while (left > 0 && rounds < max_rounds) {
        CHK(run(1));
        ++rounds;
        CHK(remaining(&left));
      }
      CHK(run(2));
    }
  } else {
    CHK(run(0));
    int rounds = 0;
    while (left > 0 && rounds < max_rounds) {
      CHK(run(1));
      ++rounds;
      CHK(remaining(&left));
    }
    CHK(run(2));
    if (use_graph && left == 0) whole_rounds = rounds;
  }
  HIPCHK(c, hipEventRecord(c->ev[6], bs));
  HIPCHK(c, hipStreamSynchronize(bs));
  if (whole_rounds > 0) {  // later solves of this shape run as one graph of this many rounds
    CHK(capture(&c->bgraph[3], [&](hipStream_t q) {
      phase_init(q);
      for (int r = 0; r < whole_rounds; ++r) phase_round(q);
      phase_out(q);
    }));
    c->bwhole_rounds = whole_rounds;
  }
  // per-configuration results
  std::vector<int> its(nconf), status(nconf);
  std::vector<double> res(nconf);
  std::vector<unsigned long long> t0(nconf), t1(nconf);
  HIPCHK(c, hipMemcpy(its.data(), st.iters, nconf * sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(status.data(), st.status, nconf * sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(res.data(), st.resid, nconf * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(t0.data(), st.t0, nconf * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(t1.data(), st.t1, nconf * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  int rate_khz = 0;
  HIPCHK(c, hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device));
  unsigned long long tmin = ~0ull;
  for (int b = 0; b < nconf; ++b) tmin = std::min(tmin, t0[b]);
  const double total_ms = ev_ms(c->ev[5], c->ev[6]);
  int rc = MBS_OK;
  for (int b = 0; b < nconf; ++b) {
    const int64_t nb = offsets[b + 1] - offsets[b];
    if (per_conf) {
      mbs_stats& o = per_conf[b];
      memset(&o, 0, sizeof o);
      o.iters = its[b];
      o.fp64_matvecs = its[b] + 1;
      o.rel_resid = res[b];
      o.t_total_ms = total_ms;
      o.pair_blocks = (double)nb * (double)(nb - 1) * (its[b] + 3);
    }
    if (latency_ms)
      latency_ms[b] = rate_khz > 0 ? (double)(t1[b] - tmin) / (double)rate_khz : total_ms;
    if (status[b] != kFinal || !(res[b] <= tol)) rc = MBS_ENOCONV;
  }
  // the caller's stream continues after the batch
  HIPCHK(c, hipEventRecord(c->ev[7], bs));
  HIPCHK(c, hipStreamWaitEvent(s, c->ev[7], 0));
  if (rc == MBS_ENOCONV) set_err(c, MBS_ENOCONV, "some configurations did not reach the tolerance");
  return rc;
}

int mbs_autotune_batched(mbs_ctx* c, int32_t nconf, const int64_t* offsets, const double* R, int32_t* chosen,
                         double* ms, void* stream) {
  CHK(begin_call(c));
  CHK(check_offsets(c, nconf, offsets));
  if (!R) return set_err(c, MBS_EINVAL, "R is required");
  hipStream_t s = (hipStream_t)stream;
  CHK(ensure_ws(c, 16));
  const int ntot = (int)offsets[nconf];
  const int64_t len = 5 * (int64_t)ntot;
  std::vector<int> off(nconf + 1);
  for (int b = 0; b <= nconf; ++b) off[b] = (int)offsets[b];
  // scratch: source records, x (zero), y, items (sized for the smallest item), offsets, status
  size_t bytes = 0;
  auto reserve = [&](size_t b) { size_t o = bytes; bytes += align256(b); return o; };
  const size_t orec = reserve((size_t)ntot * sizeof(Src8<double>)), ox = reserve(len * 8), oy = reserve(len * 8),
               oit = reserve(((size_t)ntot / 64 + nconf + 1) * sizeof(int2)), ooff = reserve((nconf + 1) * 4),
               ost = reserve((size_t)nconf * 4);
  CHK(ensure(c, c->btune, bytes / 8 + 64));
  char* base = (char*)c->btune.p;
  Src8<double>* rec = (Src8<double>*)(base + orec);
  double *x = (double*)(base + ox), *y = (double*)(base + oy);
  int2* ditems = (int2*)(base + oit);
  int *doff = (int*)(base + ooff), *dst = (int*)(base + ost);
  HIPCHK(c, hipMemcpyAsync(doff, off.data(), (nconf + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  batched_set_ints(dst, nconf, kActive, s);  // every configuration takes part
  batched_fill(x, 0.0, len, s);
  batched_pack_s(R, x, nullptr, 0, 0, rec, ntot, s);
  const int cand[3] = {64, 128, 256};
  double best = 0.0;
  int pick = 64;
  std::vector<int2> items;
  for (int k = 0; k < 3; ++k) {
    batch_items(off, nconf, cand[k], items);
    HIPCHK(c, hipMemcpyAsync(ditems, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    const int ni = (int)items.size();
    batched_p2(ditems, ni, cand[k], doff, dst, kActive, rec, x, nullptr, 0, c->ph, y, s);  // warm-up
    HIPCHK(c, hipEventRecord(c->ev[0], s));
    for (int r = 0; r < 3; ++r) batched_p2(ditems, ni, cand[k], doff, dst, kActive, rec, x, nullptr, 0, c->ph, y, s);
    HIPCHK(c, hipEventRecord(c->ev[1], s));
    HIPCHK(c, hipEventSynchronize(c->ev[1]));
    const double t = ev_ms(c->ev[0], c->ev[1]) / 3.0;
    if (ms) ms[k] = t;
    if (k == 0 || t < best) {
      best = t;
      pick = cand[k];
    }
  }
  HIPCHK(c, hipGetLastError());
  c->bitem = pick;
  if (chosen) *chosen = pick;
  return MBS_OK;
}

int mbs_autotune(mbs_ctx* c, int64_t n, const double* R, const char* cache_json, int32_t* chosen,
                 void* stream) {
  CHK(begin_call(c));
  if (n < 2 || !R) return set_err(c, MBS_EINVAL, "autotune needs n >= 2 and R");
  if (n > (int64_t)INT32_MAX / 6) return set_err(c, MBS_EINVAL, "n too large");
  hipStream_t s = (hipStream_t)stream;
  CHK(ensure_ws(c, n));
  int bucket = 0;
  while ((int64_t(1) << (bucket + 1)) <= n) ++bucket;
  char key64[64], key32[64];
  snprintf(key64, sizeof key64, "gfx950:f64:n2^%d", bucket);
  snprintf(key32, sizeof key32, "gfx950:f32:n2^%d", bucket);
  // cache: a flat JSON object of "key": value pairs
  std::vector<std::pair<std::string, double>> kv;
  if (cache_json) {
    FILE* f = fopen(cache_json, "r");
    if (f) {
      std::string txt;
      char buf[4096];
      size_t got;
      while ((got = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, got);
      fclose(f);
      size_t pos = 0;
      while ((pos = txt.find('"', pos)) != std::string::npos) {
        const size_t e = txt.find('"', pos + 1);
        if (e == std::string::npos) break;
        const std::string k = txt.substr(pos + 1, e - pos - 1);
        const size_t colon = txt.find(':', e);
        if (colon == std::string::npos) break;
        kv.emplace_back(k, strtod(txt.c_str() + colon + 1, nullptr));
        pos = txt.find_first_of(",}", colon);
        if (pos == std::string::npos) break;
      }
    }
  }
  auto lookup = [&](const char* k, int* out) {
    for (auto& p : kv)
      if (p.first == k && p.second >= 0 && p.second < kTileCount) {
        *out = (int)p.second;
        return true;
      }
    return false;
  };
  int best[2] = {0, 0};
  double best_ms[2] = {0.0, 0.0};
  const bool cached = lookup(key64, &best[0]) && lookup(key32, &best[1]);
  if (!cached) {
    const int64_t len = 5 * n;
    HIPCHK(c, hipMemsetAsync(c->xs.p, 0, len * sizeof(double), s));
    for (int prec = 0; prec < 2; ++prec) {
      double bt = 1e300;
      for (int k = 0; k < kTileCount; ++k) {
        const Tile t = kTileTable[k];
        // one warm-up launch, then the mean of three timed launches
        launch_p2(prec == 1, R, c->xs.p, c->w.p, c->part.p, c->srcbuf.p, c->orig.p, n, c->ph, t, s);
        HIPCHK(c, hipEventRecord(c->ev[6], s));
        for (int r = 0; r < 3; ++r)
          launch_p2(prec == 1, R, c->xs.p, c->w.p, c->part.p, c->srcbuf.p, c->orig.p, n, c->ph, t, s);
        HIPCHK(c, hipEventRecord(c->ev[7], s));
        HIPCHK(c, hipEventSynchronize(c->ev[7]));
        HIPCHK(c, hipGetLastError());
        const double ms = ev_ms(c->ev[6], c->ev[7]) / 3.0;
        if (ms < bt) {
          bt = ms;
          best[prec] = k;
        }
      }
      best_ms[prec] = bt;
    }
    if (cache_json) {
      bool f64 = false, f32 = false;
      for (auto& p : kv) {
        if (p.first == key64) p.second = best[0], f64 = true;
        if (p.first == key32) p.second = best[1], f32 = true;
      }
      if (!f64) kv.emplace_back(key64, best[0]);
      if (!f32) kv.emplace_back(key32, best[1]);
      char mk[96];
      snprintf(mk, sizeof mk, "%s:ms", key64);
      kv.emplace_back(mk, best_ms[0]);
      snprintf(mk, sizeof mk, "%s:ms", key32);
      kv.emplace_back(mk, best_ms[1]);
      FILE* f = fopen(cache_json, "w");
      if (f) {
        fprintf(f, "{\n");
        for (size_t k = 0; k < kv.size(); ++k)
          fprintf(f, "  \"%s\": %.17g%s\n", kv[k].first.c_str(), kv[k].second,
                  k + 1 < kv.size() ? "," : "");
        fprintf(f, "}\n");
        fclose(f);
      }
    }
  }
  c->tuned64 = best[0];
  c->tuned32 = best[1];
  apply_tiles(c);
  if (chosen) {
    chosen[0] = best[0];
    chosen[1] = best[1];
  }
  return MBS_OK;
}

int mbs_features(mbs_ctx* c, int64_t n, const double* R, const double* p, float* feat, int32_t* nbr,
                 void* stream) {
  CHK(begin_call(c));
  if (n < kNeigh + 1) return set_err(c, MBS_EINVAL, "features need n >= %d", kNeigh + 1);
  if (n > (int64_t)INT32_MAX / kMlpIn) return set_err(c, MBS_EINVAL, "n too large");
  if (!R || !p || !feat) return set_err(c, MBS_EINVAL, "R, p and feat are required");
  hipStream_t s = (hipStream_t)stream;
  CHK(check_inputs(c, s, {{R, 3 * n}}, p, n));
  int32_t* nb = nbr;
  if (!nb) {
    CHK(ensure(c, c->knn_buf, (size_t)n * kNeigh / 2 + 64));
    nb = (int32_t*)c->knn_buf.p;
  }
  CHK(knn_features(c, n, R, p, feat, nb, s));
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_features_ex(mbs_ctx* c, int64_t n, const double* R, const double* p, const double* b, float* feat,
                    int32_t* nbr, void* stream) {
  CHK(begin_call(c));
  if (n < kNeigh + 1) return set_err(c, MBS_EINVAL, "features need n >= %d", kNeigh + 1);
  if (n > (int64_t)INT32_MAX / kMlpInMax) return set_err(c, MBS_EINVAL, "n too large");
  if (!R || !p || !feat) return set_err(c, MBS_EINVAL, "R, p and feat are required");
  const bool rhs = c->mlp_set == MBS_FEATURES_GEOMETRY_RHS;
  if (rhs && !b) return set_err(c, MBS_EINVAL, "this feature set needs the right-hand side b");
  hipStream_t s = (hipStream_t)stream;
  CHK(check_inputs(c, s, {{R, 3 * n}, {rhs ? b : nullptr, 5 * n}}, p, n));
  int32_t* nb = nbr;
  if (!nb) {
    CHK(ensure(c, c->knn_buf, (size_t)n * kNeigh / 2 + 64));
    nb = (int32_t*)c->knn_buf.p;
  }
  CHK(knn_features(c, n, R, p, feat, nb, s, c->mlp_set, b));
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_warmstart_features(mbs_ctx* c, int32_t feature_set) {
  CHK(begin_call(c));
  if (feature_set != MBS_FEATURES_GEOMETRY && feature_set != MBS_FEATURES_GEOMETRY_RHS)
    return set_err(c, MBS_EINVAL, "unknown feature set %d", feature_set);
  c->mlp_set = feature_set;
  c->mlp_lay = mlp_layout(feature_set == MBS_FEATURES_GEOMETRY_RHS ? kMlpInRhs : kMlpIn);
  c->mlp_ready = false;  // the network must be initialised, set or loaded again
  return MBS_OK;
}

int mbs_warmstart_set(mbs_ctx* c, const float* params) {
  CHK(begin_call(c));
  if (!params) return set_err(c, MBS_EINVAL, "params is NULL");
  const MlpLayout& L = c->mlp_lay;
  for (int k = 0; k < L.nparam; ++k)
    if (!isfinite(params[k])) return set_err(c, MBS_EINVAL, "non-finite parameter %d", k);
  CHK(mlp_ensure(c, 16));
  MlpW W = mlp_weights(c);
  HIPCHK(c, hipMemcpy(W.w, params, L.nparam * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemset(c->mlp_m.p, 0, L.nparam * sizeof(float)));
  HIPCHK(c, hipMemset(c->mlp_v.p, 0, L.nparam * sizeof(float)));
  mlp_weights_bf16(W.w, L, W.W1, W.W2, W.W3, nullptr);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipDeviceSynchronize());
  c->adam_step = 0;
  c->mlp_ready = true;
  return MBS_OK;
}

int mbs_warmstart_init(mbs_ctx* c, uint64_t seed) {
  CHK(begin_call(c));
  // He-uniform weights U(-sqrt(6/fan_in), sqrt(6/fan_in)), zero biases
  const MlpLayout& L = c->mlp_lay;
  std::vector<float> w(L.nparam, 0.f);
  std::mt19937_64 gen(seed);
  auto fill = [&](int off, int fan_in, int count) {
    std::uniform_real_distribution<double> U(-sqrt(6.0 / fan_in), sqrt(6.0 / fan_in));
    for (int k = 0; k < count; ++k) w[off + k] = (float)U(gen);
  };
  fill(L.offW1, L.in, L.in * kMlpHid);
  fill(L.offW2, kMlpHid, kMlpHid * kMlpHid);
  fill(L.offW3, kMlpHid, kMlpHid * kMlpOut);
  return mbs_warmstart_set(c, w.data());
}

int mbs_warmstart_get(mbs_ctx* c, float* params) {
  CHK(begin_call(c));
  if (!params) return set_err(c, MBS_EINVAL, "params is NULL");
  if (!c->mlp_ready) return set_err(c, MBS_EUNSUPPORTED, "no warm-start network in this context");
  HIPCHK(c, hipMemcpy(params, c->mlp_w.p, c->mlp_lay.nparam * sizeof(float), hipMemcpyDeviceToHost));
  return MBS_OK;
}

int mbs_warmstart_forward(mbs_ctx* c, int64_t m, const float* feat, float* out, void* stream) {
  CHK(begin_call(c));
  if (m < 1 || !feat || !out) return set_err(c, MBS_EINVAL, "m >= 1, feat and out are required");
  if (m > (int64_t)INT32_MAX / kMlpInMax) return set_err(c, MBS_EINVAL, "m too large");
  if (!c->mlp_ready) return set_err(c, MBS_EUNSUPPORTED, "no warm-start network in this context");
  hipStream_t s = (hipStream_t)stream;
  CHK(mlp_forward(c, m, feat, out, s));
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_warmstart_grad(mbs_ctx* c, int64_t m, const float* feat, const float* target, float* grad,
                       double* loss, void* stream) {
  CHK(begin_call(c));
  if (m < 1 || m > kChunkRows || !feat || !target || !grad)
    return set_err(c, MBS_EINVAL, "1 <= m <= %d; feat, target and grad are required", kChunkRows);
  if (!c->mlp_ready) return set_err(c, MBS_EUNSUPPORTED, "no warm-start network in this context");
  hipStream_t s = (hipStream_t)stream;
  const int rows = (int)m, rp = ceil16(rows);
  CHK(mlp_ensure(c, rp));
  MlpWs ws = mlp_carve(c, rp);
  double* lp = (double*)c->mlp_loss.p;
  mlp_forward_rows(c, feat, nullptr, rows, ws, s);
  mlp_backward_rows(c, target, nullptr, rows, ws, lp, s);
  HIPCHK(c, hipGetLastError());
  const int nb = mlp_mse_blocks(rp);
  std::vector<double> parts(nb);
  HIPCHK(c, hipMemcpyAsync(parts.data(), lp, nb * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(grad, c->mlp_g.p, c->mlp_lay.nparam * sizeof(float), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  double sum = 0.0;
  for (double v : parts) sum += v;
  if (loss) *loss = sum / ((double)rows * kMlpOut);
  return MBS_OK;
}

int mbs_warmstart_train(mbs_ctx* c, int64_t m, const float* feat, const float* target, int32_t epochs,
                        int32_t batch, double lr, uint64_t seed, double* loss_hist, void* stream) {
  CHK(begin_call(c));
  if (m < 1 || !feat || !target) return set_err(c, MBS_EINVAL, "m >= 1, feat and target are required");
  if (m > (int64_t)INT32_MAX / kMlpInMax) return set_err(c, MBS_EINVAL, "m too large");
  if (epochs < 0 || batch < 16 || batch > kChunkRows || !(lr > 0.0))
    return set_err(c, MBS_EINVAL, "need epochs >= 0, 16 <= batch <= %d, lr > 0", kChunkRows);
  if (!c->mlp_ready) return set_err(c, MBS_EUNSUPPORTED, "initialise the network first");
  hipStream_t s = (hipStream_t)stream;
  const int bp = ceil16(batch);
  CHK(mlp_ensure(c, bp));
  const int64_t nbatch = (m + batch - 1) / batch;
  const int nbl = mlp_mse_blocks(bp);
  CHK(ensure(c, c->mlp_loss, (size_t)nbatch * nbl + 64));
  CHK(ensure(c, c->mlp_idx, (size_t)m / 2 + 64));
  MlpWs ws = mlp_carve(c, bp);
  MlpW W = mlp_weights(c);
  int32_t* didx = (int32_t*)c->mlp_idx.p;
  std::vector<int32_t> perm(m);
  std::mt19937_64 gen(seed);
  std::vector<double> parts((size_t)nbatch * nbl);
  for (int e = 0; e < epochs; ++e) {
    for (int64_t k = 0; k < m; ++k) perm[k] = (int32_t)k;
    for (int64_t k = m - 1; k > 0; --k) {  // Fisher-Yates
      std::uniform_int_distribution<int64_t> U(0, k);
      std::swap(perm[k], perm[U(gen)]);
    }
    HIPCHK(c, hipMemcpyAsync(didx, perm.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemsetAsync(c->mlp_loss.p, 0, (size_t)nbatch * nbl * sizeof(double), s));
    for (int64_t bi = 0; bi < nbatch; ++bi) {
      const int rows = (int)std::min<int64_t>(batch, m - bi * batch);
      const int32_t* idx = didx + bi * batch;
      mlp_forward_rows(c, feat, idx, rows, ws, s);
      mlp_backward_rows(c, target, idx, rows, ws, (double*)c->mlp_loss.p + bi * nbl, s);
      mlp_adam(W.w, (const float*)c->mlp_g.p, (float*)c->mlp_m.p, (float*)c->mlp_v.p, c->mlp_lay.nparam,
               (float)lr, 0.9f, 0.999f, 1e-8f, ++c->adam_step, s);
      mlp_weights_bf16(W.w, c->mlp_lay, W.W1, W.W2, W.W3, s);
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(parts.data(), c->mlp_loss.p, parts.size() * sizeof(double),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    double sum = 0.0;
    for (double v : parts) sum += v;
    if (loss_hist) loss_hist[e] = sum / ((double)m * kMlpOut);
  }
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_warmstart_save(mbs_ctx* c, const char* path) {
  CHK(begin_call(c));
  if (!path) return set_err(c, MBS_EINVAL, "path is NULL");
  if (!c->mlp_ready) return set_err(c, MBS_EUNSUPPORTED, "no warm-start network in this context");
  const int np = c->mlp_lay.nparam;
  std::vector<float> w(np);
  HIPCHK(c, hipMemcpy(w.data(), c->mlp_w.p, np * sizeof(float), hipMemcpyDeviceToHost));
  FILE* f = fopen(path, "wb");
  if (!f) return set_err(c, MBS_EINVAL, "cannot write %s", path);
  const uint32_t hdr[4] = {0x5753424Du /* "MBSW" */, 2u, (uint32_t)np, (uint32_t)c->mlp_set};
  const bool ok = fwrite(hdr, sizeof hdr, 1, f) == 1 && fwrite(w.data(), sizeof(float), np, f) == (size_t)np;
  fclose(f);
  return ok ? MBS_OK : set_err(c, MBS_EINVAL, "short write to %s", path);
}

int mbs_warmstart_load(mbs_ctx* c, const char* path) {
  CHK(begin_call(c));
  if (!path) return set_err(c, MBS_EINVAL, "path is NULL");
  FILE* f = fopen(path, "rb");
  if (!f) return set_err(c, MBS_EINVAL, "cannot read %s", path);
  uint32_t hdr[3] = {0, 0, 0};
  uint32_t set = MBS_FEATURES_GEOMETRY;
  bool ok = fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == 0x5753424Du && (hdr[1] == 1u || hdr[1] == 2u);
  if (ok && hdr[1] == 2u) ok = fread(&set, sizeof set, 1, f) == 1;  // version 1: the 80-input network
  ok = ok && (set == (uint32_t)MBS_FEATURES_GEOMETRY || set == (uint32_t)MBS_FEATURES_GEOMETRY_RHS);
  const MlpLayout L = mlp_layout(set == (uint32_t)MBS_FEATURES_GEOMETRY_RHS ? kMlpInRhs : kMlpIn);
  std::vector<float> w(ok ? L.nparam : 0);
  ok = ok && hdr[2] == (uint32_t)L.nparam && fread(w.data(), sizeof(float), L.nparam, f) == (size_t)L.nparam;
  fclose(f);
  if (!ok) return set_err(c, MBS_EINVAL, "%s is not a warm-start weight file", path);
  CHK(mbs_warmstart_features(c, (int32_t)set));
  return mbs_warmstart_set(c, w.data());
}

int mbs_initial_guess(mbs_ctx* c, int64_t n, const double* R, const double* p, const double* v2s,
                      const double* v3t, const double* Fe, const double* Te, int32_t guess,
                      double* sigma0, void* stream) {
  CHK(begin_call(c));
  CHK(refuse_plane(c, "mbs_initial_guess"));
  if (n < 1 || !R || !sigma0) return set_err(c, MBS_EINVAL, "n >= 1, R and sigma0 are required");
  if (n > (int64_t)INT32_MAX / kMlpIn) return set_err(c, MBS_EINVAL, "n too large");
  if (guess != MBS_GUESS_ZERO && guess != MBS_GUESS_DIAG && guess != MBS_GUESS_LEARNED)
    return set_err(c, MBS_EINVAL, "guess must be MBS_GUESS_ZERO, _DIAG or _LEARNED");
  if (guess == MBS_GUESS_LEARNED) CHK(check_learned(c, n, p));
  CHK(check_aliasing(c, {{"sigma0", sigma0, 5 * n}},
                     {{"R", R, 3 * n}, {"p", p, 3 * n}, {"v2s", v2s, 5 * n}, {"v3t", v3t, 3 * n},
                      {"Fe", Fe, 3 * n}, {"Te", Te, 3 * n}}));
  hipStream_t s = (hipStream_t)stream;
  CHK(ensure_ws(c, n));
  if (guess == MBS_GUESS_LEARNED) CHK(check_inputs(c, s, {{R, 3 * n}}, p, n));
  launch_p1(R, v2s, v3t, Fe ? Fe : c->zeros.p, Te, c->b.p, c->part.p, n, c->ph, c->tile_pass, s);
  if (guess == MBS_GUESS_ZERO)
    launch_axpby(0.0, c->b.p, 0.0, sigma0, 5 * n, s);
  else if (guess == MBS_GUESS_DIAG)
    launch_axpby(c->ph.gamma, c->b.p, 0.0, sigma0, 5 * n, s);
  else
    CHK(learned_guess(c, n, R, p, c->b.p, sigma0, s));
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_warmstart_target(mbs_ctx* c, int64_t n, const double* R, const double* v2s, const double* v3t,
                         const double* Fe, const double* Te, const double* Sigma, float* target,
                         void* stream) {
  CHK(begin_call(c));
  CHK(refuse_plane(c, "mbs_warmstart_target"));
  if (n < 1 || !R || !Sigma || !target) return set_err(c, MBS_EINVAL, "n >= 1, R, Sigma, target required");
  if (n > (int64_t)INT32_MAX / kMlpIn) return set_err(c, MBS_EINVAL, "n too large");
  hipStream_t s = (hipStream_t)stream;
  CHK(ensure_ws(c, n));
  launch_p1(R, v2s, v3t, Fe ? Fe : c->zeros.p, Te, c->b.p, c->part.p, n, c->ph, c->tile_pass, s);
  launch_target(Sigma, c->b.p, c->ph.gamma, 5 * n, target, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_precond_apply(mbs_ctx* c, int64_t n, const double* R, const double* x, double* y, void* stream) {
  CHK(begin_call(c));
  if (n < 1 || !R || !x || !y) return set_err(c, MBS_EINVAL, "n >= 1, R, x and y are required");
  if (n > (int64_t)INT32_MAX / 6) return set_err(c, MBS_EINVAL, "n too large");
  CHK(check_aliasing(c, {{"y", y, 5 * n}}, {{"R", R, 3 * n}, {"x", x, 5 * n}}));
  if (!(c->prm.near_cutoff > 0.0)) return set_err(c, MBS_EINVAL, "params.near_cutoff must be > 0");
  hipStream_t s = (hipStream_t)stream;
  CHK(ensure_ws(c, n));
  CHK(near_prepare(c, n, R, s));
  near_apply(c, n, R, x, y, s);
  c->near_ready = false;
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}


int mbs_matvec_r3(mbs_ctx* c, int64_t n, const double* R, const double* x, double* y, void* stream) {
  CHK(begin_call(c));
  CHK(refuse_plane(c, "the rank-3 entry points"));
  CHK(r3_check_n(c, n));
  if (!R || !x || !y) return set_err(c, MBS_EINVAL, "R, x and y are required");
  CHK(check_aliasing(c, {{"y", y, 20 * n}}, {{"R", R, 3 * n}, {"x", x, 20 * n}}));
  hipStream_t s = (hipStream_t)stream;
  R3Ws ws;
  CHK(r3_workspace(c, n, &ws));
  launch_rank3(0, R, x, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, y, nullptr, nullptr,
               ws.part, n, c->ph, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_rhs_r3(mbs_ctx* c, int64_t n, const double* R, const double* v2s, const double* v3t, const mbs_slip_ex* ex,
               const double* Fe, const double* Te, double* b, void* stream) {
  CHK(begin_call(c));
  CHK(refuse_plane(c, "the rank-3 entry points"));
  CHK(r3_check_n(c, n));
  if (!R || !b) return set_err(c, MBS_EINVAL, "R and b are required");
  const HighSlip hi = high_of(ex);
  CHK(check_aliasing(c, {{"b", b, 20 * n}},
                     {{"R", R, 3 * n}, {"v2s", v2s, 5 * n}, {"v3t", v3t, 3 * n}, {"Fe", Fe, 3 * n},
                      {"Te", Te, 3 * n}, {"gam", hi.gam, 10 * n}, {"psi", hi.psi, 5 * n}, {"lam", hi.lam, 10 * n}}));
  hipStream_t s = (hipStream_t)stream;
  R3Ws ws;
  CHK(r3_workspace(c, n, &ws));
  launch_rank3(1, R, nullptr, nullptr, v2s, v3t, hi.gam, hi.psi, hi.lam, Fe, Te, b, nullptr, nullptr, ws.part, n,
               c->ph, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_outputs_r3(mbs_ctx* c, int64_t n, const double* R, const double* v1s, const double* v2s,
                   const mbs_slip_ex* ex, const double* Fe, const double* Te, const double* x, double* V, double* W,
                   double* S, void* stream) {
  CHK(begin_call(c));
  CHK(refuse_plane(c, "the rank-3 entry points"));
  CHK(r3_check_n(c, n));
  if (!R || !x || !V || !W) return set_err(c, MBS_EINVAL, "R, x, V and W are required");
  const HighSlip hi = high_of(ex);
  CHK(check_aliasing(c, {{"V", V, 3 * n}, {"W", W, 3 * n}, {"S", S, 5 * n}},
                     {{"R", R, 3 * n}, {"v1s", v1s, 3 * n}, {"v2s", v2s, 5 * n}, {"Fe", Fe, 3 * n},
                      {"Te", Te, 3 * n}, {"x", x, 20 * n}, {"lam", hi.lam, 10 * n}}));
  hipStream_t s = (hipStream_t)stream;
  R3Ws ws;
  CHK(r3_workspace(c, n, &ws));
  launch_rank3(2, R, x, v1s, v2s, nullptr, nullptr, nullptr, hi.lam, Fe, Te, V, W, S, ws.part, n, c->ph, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_precond_apply_r3(mbs_ctx* c, int64_t n, const double* R, const double* x, double* y, void* stream) {
  CHK(begin_call(c));
  CHK(refuse_plane(c, "the rank-3 entry points"));
  CHK(r3_check_n(c, n));
  if (!R || !x || !y) return set_err(c, MBS_EINVAL, "R, x and y are required");
  CHK(check_aliasing(c, {{"y", y, 20 * n}}, {{"R", R, 3 * n}, {"x", x, 20 * n}}));
  if (!(c->prm.near_cutoff > 0.0)) return set_err(c, MBS_EINVAL, "params.near_cutoff must be > 0");
  hipStream_t s = (hipStream_t)stream;
  R3Ws ws;
  CHK(r3_workspace(c, n, &ws));
  CHK(near_prepare(c, n, R, s));
  r3_precond(c, n, R, x, y, ws, s);
  c->near_ready = false;
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  return MBS_OK;
}

int mbs_solve_r3(mbs_ctx* c, int64_t n, const double* R, const double* v1s, const double* v2s, const double* v3t,
                 const mbs_slip_ex* ex, const double* Fe, const double* Te, const double* x0, double* V, double* W,
                 double* S, double* x, mbs_stats* st, void* stream) {
  CHK(begin_call(c));
  CHK(refuse_plane(c, "the rank-3 entry points"));
  CHK(r3_check_n(c, n));
  if (!R || !V || !W || !S) return set_err(c, MBS_EINVAL, "R, V, W and S are required");
  const HighSlip hi = high_of(ex);
  CHK(check_aliasing(c, {{"V", V, 3 * n}, {"W", W, 3 * n}, {"S", S, 5 * n}, {"x", x, 20 * n}},
                     {{"R", R, 3 * n}, {"v1s", v1s, 3 * n}, {"v2s", v2s, 5 * n}, {"v3t", v3t, 3 * n},
                      {"Fe", Fe, 3 * n}, {"Te", Te, 3 * n}, {"x0", x0, 20 * n}, {"gam", hi.gam, 10 * n},
                      {"psi", hi.psi, 5 * n}, {"lam", hi.lam, 10 * n}}));
  hipStream_t s = (hipStream_t)stream;
  R3Ws ws;
  CHK(r3_workspace(c, n, &ws));
  CHK(check_inputs(c, s, {{R, 3 * n}, {v1s, 3 * n}, {v2s, 5 * n}, {v3t, 3 * n}, {Fe, 3 * n}, {Te, 3 * n},
                          {x0, 20 * n}, {hi.gam, 10 * n}, {hi.psi, 5 * n}, {hi.lam, 10 * n}},
                   nullptr, n));
  if (c->prm.check_overlap) {
    double md = 0.0;
    CHK(check_overlap(c, n, R, s, &md));
    if (md < 2.0 * c->prm.a)
      return set_err(c, MBS_EOVERLAP, "spheres overlap: minimum centre distance %.6g < 2a", md);
  }
  const int64_t len = 20 * n;
  Counters cnt;
  Small sm = small_of(c);
  c->npend = 0;
  c->t_op[0] = c->t_op[1] = 0.0;
  HIPCHK(c, hipEventRecord(c->ev[0], s));
  launch_rank3(1, R, nullptr, nullptr, v2s, v3t, hi.gam, hi.psi, hi.lam, Fe, Te, ws.b, nullptr, nullptr, ws.part, n,
               c->ph, s);
  cnt.pairs += (double)n * (double)(n - 1);
  HIPCHK(c, hipEventRecord(c->ev[1], s));
  norm2(c, ws.b, len, sm.bnorm2, s);
  CHK(read_status(c, sm.bnorm2, 1, s));
  const double bnorm = sqrt(c->h_status[0]);
  // start: x0 if given, else the one-body guess D^{-1} b (params.guess = MBS_GUESS_DIAG) or zero
  const bool diag = !x0 && c->prm.guess == MBS_GUESS_DIAG;
  if (x0)
    launch_copy(x0, ws.x, len, s);
  else if (diag)
    launch_rank3_diag(ws.b, n, c->ph.gamma, ws.x, s);
  else
    launch_axpby(0.0, ws.b, 0.0, ws.x, len, s);
  const bool x_zero = !x0 && !diag;
  double resid = 0.0, rel = 0.0;
  int rc = MBS_OK;
  const bool pc = c->prm.near_cutoff > 0.0 && n > 1;
  if (bnorm == 0.0 && x_zero) {
    rel = 0.0;  // x = 0 solves the system exactly
  } else {
    if (pc) CHK(near_prepare(c, n, R, s));
    CHK(r3_gmres(c, n, R, ws, x_zero, pc, c->prm.tol * bnorm, c->prm.max_iter, &resid, cnt, s));
    c->near_ready = false;
    rel = bnorm > 0.0 ? resid / bnorm : resid;
    if (!(rel <= c->prm.tol)) rc = MBS_ENOCONV;
  }
  HIPCHK(c, hipEventRecord(c->ev[2], s));
  launch_rank3(2, R, ws.x, v1s, v2s, nullptr, nullptr, nullptr, hi.lam, Fe, Te, V, W, S, ws.part, n, c->ph, s);
  cnt.pairs += (double)n * (double)(n - 1);
  if (x) launch_copy(ws.x, x, len, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipEventRecord(c->ev[3], s));
  HIPCHK(c, hipStreamSynchronize(s));
  harvest_ops(c);
  if (st) {
    memset(st, 0, sizeof(*st));
    st->iters = cnt.iters;
    st->fp64_matvecs = cnt.f64;
    st->rel_resid = rel;
    st->t_rhs_ms = ev_ms(c->ev[0], c->ev[1]);
    st->t_iter_ms = ev_ms(c->ev[1], c->ev[2]);
    st->t_out_ms = ev_ms(c->ev[2], c->ev[3]);
    st->t_total_ms = ev_ms(c->ev[0], c->ev[3]);
    st->t_op64_ms = c->t_op[0];
    st->pair_blocks = cnt.pairs;
  }
  if (rc == MBS_ENOCONV)
    set_err(c, MBS_ENOCONV, "no convergence: relative residual %.3e after %d iterations", rel, cnt.iters);
  return rc;
}

}  // extern "C"
