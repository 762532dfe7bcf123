// Host build of the generated periodic arithmetic (paper_1411_0278_amd/csrc/mbs_periodic_gen.h) for
// the CPU tests: each entry evaluates one generated function over n separations or wave vectors.
#include <cmath>
#define __device__
#define __host__
#define __forceinline__ inline
#include "mbs_periodic_gen.h"

extern "C" {
// x [n x 3] separations; outputs start at zero
void ev_real(int which, int n, const double* x, double xi, double a2, const double* f, const double* t,
             const double* s, const double* q, double* o1, double* o2) {
  for (int p = 0; p < n; ++p) {
    const double* d = x + 3 * p;
    const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double ri = 1.0 / r, ec = std::erfc(xi * r), ex = std::exp(-xi * xi * r * r);
    if (which == 0) {
      for (int c = 0; c < 5; ++c) o1[5 * p + c] = 0.0;
      mbs::per_real_strain_s(d[0], d[1], d[2], ri, ec, ex, xi, a2, s + 5 * p, o1 + 5 * p);
    } else if (which == 1) {
      for (int c = 0; c < 5; ++c) o1[5 * p + c] = 0.0;
      mbs::per_real_strain_ftq(d[0], d[1], d[2], ri, ec, ex, xi, a2, f + 3 * p, t + 3 * p, q + 3 * p, o1 + 5 * p);
    } else if (which == 2) {
      for (int c = 0; c < 3; ++c) o1[3 * p + c] = o2[3 * p + c] = 0.0;
      mbs::per_real_motion_ftsq(d[0], d[1], d[2], ri, ec, ex, xi, a2, f + 3 * p, t + 3 * p, s + 5 * p, q + 3 * p,
                                o1 + 3 * p, o2 + 3 * p);
    } else {
      for (int c = 0; c < 3; ++c) o1[3 * p + c] = 0.0;
      mbs::per_real_flow_ftsq(d[0], d[1], d[2], ri, ec, ex, xi, a2, f + 3 * p, t + 3 * p, s + 5 * p, q + 3 * p,
                              o1 + 3 * p);
    }
  }
}
// k [n x 3]; the coefficients' real and imaginary parts interleaved per wave vector as
// (fr, fi, tr, ti, sr, si, qr, qi); outputs real and imaginary parts
void ev_hat(int which, int n, const double* k, double a2, const double* fr, const double* fi, const double* tr,
            const double* ti, const double* sr, const double* si, const double* qr, const double* qi, double* outr,
            double* outi) {
  for (int p = 0; p < n; ++p) {
    const double* kv = k + 3 * p;
    const double ik2 = 1.0 / (kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2]);
    if (which == 0)
      mbs::per_hat_strain_s(kv[0], kv[1], kv[2], ik2, a2, sr + 5 * p, si + 5 * p, outr + 5 * p, outi + 5 * p);
    else if (which == 1)
      mbs::per_hat_strain_ftq(kv[0], kv[1], kv[2], ik2, a2, fr + 3 * p, fi + 3 * p, tr + 3 * p, ti + 3 * p, qr + 3 * p,
                              qi + 3 * p, outr + 5 * p, outi + 5 * p);
    else if (which == 2)
      mbs::per_hat_motion_ftsq(kv[0], kv[1], kv[2], ik2, a2, fr + 3 * p, fi + 3 * p, tr + 3 * p, ti + 3 * p,
                               sr + 5 * p, si + 5 * p, qr + 3 * p, qi + 3 * p, outr + 6 * p, outi + 6 * p);
    else
      mbs::per_hat_flow_ftsq(kv[0], kv[1], kv[2], ik2, a2, fr + 3 * p, fi + 3 * p, tr + 3 * p, ti + 3 * p,
                             sr + 5 * p, si + 5 * p, qr + 3 * p, qi + 3 * p, outr + 3 * p, outi + 3 * p);
  }
}
// radial functions (al, be, ga) of the screened stresslet strain at distances r [n]
void ev_es_radial(int n, const double* r, double xi, double a2, double* abg) {
  for (int p = 0; p < n; ++p)
    mbs::per_real_es_radial(1.0 / r[p], std::erfc(xi * r[p]), std::exp(-xi * xi * r[p] * r[p]), xi, a2, abg + 3 * p);
}
// radial functions of the right-hand side's strain (5) and of the outputs' motion (12) at distances r [n]
void ev_ftq_radial(int n, const double* r, double xi, double a2, double* rf) {
  for (int p = 0; p < n; ++p)
    mbs::per_real_ftq_radial(1.0 / r[p], std::erfc(xi * r[p]), std::exp(-xi * xi * r[p] * r[p]), xi, a2, rf + 5 * p);
}
void ev_motion_radial(int n, const double* r, double xi, double a2, double* rm) {
  for (int p = 0; p < n; ++p)
    mbs::per_real_motion_radial(1.0 / r[p], std::erfc(xi * r[p]), std::exp(-xi * xi * r[p] * r[p]), xi, a2,
                                rm + 12 * p);
}
void ev_flow_radial(int n, const double* r, double xi, double a2, double* rw) {
  for (int p = 0; p < n; ++p)
    mbs::per_real_flow_radial(1.0 / r[p], std::erfc(xi * r[p]), std::exp(-xi * xi * r[p] * r[p]), xi, a2, rw + 7 * p);
}
void ev_self(double xi, double a2, double* out) {
  out[0] = mbs::per_self_es(xi, a2);
  out[1] = mbs::per_self_uf(xi, a2);
  out[2] = mbs::per_self_ud(xi, a2);
  out[3] = mbs::per_self_wt(xi, a2);
}
}
