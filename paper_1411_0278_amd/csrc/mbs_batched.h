// Batched lockstep solver: launchers and per-configuration state (internal to libmbstokes).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mbs_internal.h"
#include "mbs_pair.h"

namespace mbs {

// per-configuration status words
constexpr int kActive = 1;     // inside an Arnoldi cycle
constexpr int kCycleDone = 2;  // cycle ended: update the iterate and check the true residual
constexpr int kFinal = 3;      // converged (or out of iterations)
constexpr int kRestart = 4;    // true residual short of the tolerance: restarts (Arnoldi step 0) as soon
                               // as no configuration is inside a cycle (the step index is shared)

struct BatchState {  // device arrays indexed by configuration (stride m+2 or (m+1)^2 where noted)
  double *H, *cs, *sn, *g, *y, *h1, *h2, *nsq, *bnorm, *hk1, *resid;
  int *status, *kend, *iters;
  unsigned long long *t0, *t1;
};

// near-field lists within each configuration (pairs 2a <= r < rc, first kNearCap in index order)
void batched_near_build(const int2* items, int nitems, int item, const int* off, const double* R, double rmin,
                        double rc, int* cnt, int* list, hipStream_t s);
void batched_pack_f(const double* R, const double* Fe, const double* Te, const double* D,
                    const Phys& ph, RecF* rec, int ntot, hipStream_t s);
void batched_p1(const int2* items, int nitems, int item, const int* off, const RecF* rec, const double* v2s,
                bool has_t, bool has_d, const Phys& ph, double* b, hipStream_t s);
void batched_pack_s(const double* R, const double* X, const int* kdev, int maxk, int64_t ld,
                    Src8<double>* src, int ntot, hipStream_t s);
void batched_p2(const int2* items, int nitems, int item, const int* off, const int* status, int want,
                const Src8<double>* src, const double* X, const int* kdev, int64_t ld, const Phys& ph,
                double* y, hipStream_t s);
void batched_pack_o(const double* R, const double* Fe, const double* Te, const double* Sig,
                    const double* D, const Phys& ph, RecO* rec, int ntot, hipStream_t s);
void batched_p3(const int2* items, int nitems, int item, const int* off, const RecO* rec, bool has_t, bool has_d,
                const Phys& ph, const double* v1s, const double* v2s, const double* Fe,
                const double* Te, const double* Sig, double* V, double* W, double* S, double* SigOut,
                hipStream_t s);
void batched_dots(const double* V, int64_t ld, const int* kdev, int nv_fixed, const double* w,
                  const int* off, const int* status, int want, double* h, int hstride, int nconf,
                  hipStream_t s);
void batched_axpy(const double* V, int64_t ld, const int* kdev, const int* nvb, int nv_fixed,
                  const double* h, int hstride, double sign, const int* cid, const int* status,
                  int want, double* w, int64_t len, hipStream_t s);
void batched_givens(const BatchState& b, int nconf, int m, const int* kdev, double tol, int max_iter,
                    hipStream_t s);
void batched_scale(const double* w, const double* hk1, const int* cid, const int* status, double* V,
                   int64_t ld, const int* kdev, int64_t len, hipStream_t s);
void batched_inc(int* kdev, hipStream_t s);
void batched_set_int(int* p, int v, hipStream_t s);
void batched_fill(double* x, double v, int64_t len, hipStream_t s);
void batched_set_ints(int* p, int n, int v, hipStream_t s);
void batched_backsolve(const BatchState& b, int nconf, int m, hipStream_t s);
void batched_resid(const double* bv, const double* w, const int* cid, const int* status, double* r,
                   int64_t len, hipStream_t s);
void batched_check(const BatchState& b, int nconf, int m, double tol, int max_iter, hipStream_t s);
void batched_init(const BatchState& b, int nconf, int m, hipStream_t s);
void batched_start(const double* r, const double* hk1, const int* cid, const int* status, int want,
                   double* V0, int64_t len, hipStream_t s);
void batched_count(const int* status, int nconf, int want, int* out, hipStream_t s);
// configurations whose status is not `unwanted` -> out[0]
void batched_count_not(const int* status, int nconf, int unwanted, int* out, hipStream_t s);
// if no configuration is inside a cycle: waiting restarts become active and the step index is reset
void batched_gate(int* status, int nconf, int* kdev, hipStream_t s);

}  // namespace mbs
