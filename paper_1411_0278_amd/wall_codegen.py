"""Writes csrc/mbs_wall_gen.h: the image-part arithmetic of a plane no-slip wall, per pair.

Run from the repository root after changing the derivation (the header is committed; the library
build only compiles it):

    python -m paper_1411_0278_amd.wall_codegen

Blake's solution for a point force at height h above a no-slip wall z = 0 (Proc. Camb. Phil. Soc.
70, 303 (1971)) adds to the Oseen tensor G(x - y) an image part at the source's mirror point
y* = (y_1, y_2, -h). With R = x - y*, M = diag(1, 1, -1) and the identities G_ij = 2 delta_ij / R -
d_i d_j R, R_i / R^3 = -d_i (1/R), that image part is written here through the two scalar functions
1/R and R = |R| only:

    H_ij = -(2 delta_ij / R - d_i d_j R) - 2 h M_jk d_k (2 delta_i3 / R - d_i d_3 R)
           - 2 h^2 M_jk d_k d_i (1/R).

A source sphere's flow through H takes its surface moments against H in the source point
(derivatives in y, finite-size operators F^l_y = 1 + a^2/(4l+6) lap_y); as functions of (R, h),
d/dy_1 = -d/dR_1, d/dy_2 = -d/dR_2, d/dy_3 = d/dR_3 + d/dh. Per unit of the pre-scaled source
coefficients (f = P F, t = P T, s = P Sigma in the orthonormal 5-basis, q = (a^5/20) d, P =
1/(8 pi eta)):

    u_i = F^0_y H_ij f_j + (1/2) eps_klj F^1_y dH_ij/dy_l t_k - F^1_y dH_ij/dy_k s_jk - lap_y H_ij q_j

and the receiver's projections at its centre are U = F^0_x u, W = (1/2) curl u,
E = sym grad F^1_x u (5-basis). Four device functions accumulate, for one (receiver, source) pair
given R, h, ri = 1/|R| and a2 = a^2:

    wall_strain_s      e[5] += E of s             (the operator's image part)
    wall_strain_ftq    e[5] += E of f, t, q       (the right-hand side's)
    wall_motion_ftsq   u[3] += U, w[3] += W of f, t, s, q   (the outputs')
    wall_flow_ftsq     u[3] += u of f, t, s, q at a field point (no receiver operator)

The polynomial in R, h and ri is reduced with R1^2 = R^2 - R2^2 - R3^2, grouped by source
coefficient and common subexpressions are shared within each function.
"""
from __future__ import annotations

import os
import sys

import sympy as sp
from sympy.printing.c import C99CodePrinter

Q1, Q2, Q3 = sp.symbols("R1 R2 R3", real=True)
H, RN, A2 = sp.symbols("h rn a2", positive=True)
RI = sp.symbols("ri", positive=True)
_Q = (Q1, Q2, Q3)
_MD = (1, 1, -1)
_S2, _S6 = 1 / sp.sqrt(2), 1 / sp.sqrt(6)
# orthonormal 5-basis of symmetric traceless 3 x 3 tensors (the library's layout)
_B5 = (
    ((_S2, 0, 0), (0, -_S2, 0), (0, 0, 0)),
    ((-_S6, 0, 0), (0, -_S6, 0), (0, 0, 2 * _S6)),
    ((0, _S2, 0), (_S2, 0, 0), (0, 0, 0)),
    ((0, 0, _S2), (0, 0, 0), (_S2, 0, 0)),
    ((0, 0, 0), (0, 0, _S2), (0, _S2, 0)),
)


def _red(f):
    """Expanded, with R1^2 replaced by rn^2 - R2^2 - R3^2."""
    f = sp.expand(f)
    f = f.replace(lambda e: e.is_Pow and e.base == Q1 and e.exp.is_Integer and e.exp >= 2,
                  lambda e: Q1 ** (int(e.exp) % 2) * (RN ** 2 - Q2 ** 2 - Q3 ** 2) ** (int(e.exp) // 2))
    return sp.expand(f)


def _dq(f, i):  # d/dR_i (rn = |R|)
    return _red(sp.diff(f, _Q[i]) + _Q[i] / RN * sp.diff(f, RN))


def _dsrc(f, i):  # d/dy_i at fixed field point
    return _red(-_dq(f, i)) if i < 2 else _red(_dq(f, 2) + sp.diff(f, H))


def _lap_field(f):
    return _red(sum(_dq(_dq(f, i), i) for i in range(3)))


def _lap_src(f):
    return _red(sum(_dsrc(_dsrc(f, i), i) for i in range(3)))


def blake_image():
    """H_ij through 1/R and R (module docstring)."""
    inv, dist = 1 / RN, RN
    kd = lambda i, j: int(i == j)  # noqa: E731
    Hm = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            g = 2 * kd(i, j) * inv - _dq(_dq(dist, i), j)
            doublet = 2 * kd(i, 2) * inv - _dq(_dq(dist, i), 2)
            source = _dq(inv, i)
            Hm[i][j] = _red(-g - 2 * H * _MD[j] * _dq(doublet, j) - 2 * H ** 2 * _MD[j] * _dq(source, j))
    return Hm


def _eps(k, l, j):
    return int(sp.LeviCivita(k, l, j))


def source_flows(Hm, f, t, s, q):
    """u_i of the pre-scaled coefficients f, t, q (3-vectors) and s (5-basis), any may be None."""
    u = [0, 0, 0]
    Sc = None
    if s is not None:
        Sc = [[sum(s[c] * _B5[c][j][k] for c in range(5)) for k in range(3)] for j in range(3)]
    for i in range(3):
        acc = 0
        if f is not None:
            g = sum(Hm[i][j] * f[j] for j in range(3))
            acc += g + A2 / 6 * _lap_src(g)
        if t is not None:
            g = sp.Rational(1, 2) * sum(_eps(k, l, j) * _dsrc(Hm[i][j], l) * t[k]
                                        for k in range(3) for l in range(3) for j in range(3) if _eps(k, l, j))
            acc += g + A2 / 10 * _lap_src(g)
        if s is not None:
            g = -sum(_dsrc(Hm[i][j], k) * Sc[j][k] for j in range(3) for k in range(3) if Sc[j][k] != 0)
            acc += g + A2 / 10 * _lap_src(g)
        if q is not None:
            acc += -sum(_lap_src(Hm[i][j]) * q[j] for j in range(3))
        u[i] = _red(acc)
    return u


def strain5(u):
    v = [_red(ui + A2 / 10 * _lap_field(ui)) for ui in u]
    return [_red(sum(_B5[c][i][j] * sp.Rational(1, 2) * (_dq(v[i], j) + _dq(v[j], i))
                     for i in range(3) for j in range(3) if _B5[c][i][j] != 0)) for c in range(5)]


def motion(u):
    U = [_red(ui + A2 / 6 * _lap_field(ui)) for ui in u]
    W = [_red(sp.Rational(1, 2) * (_dq(u[(i + 2) % 3], (i + 1) % 3) - _dq(u[(i + 1) % 3], (i + 2) % 3)))
         for i in range(3)]
    return U, W


class _Printer(C99CodePrinter):
    """Integer powers as products; no pow()."""

    def _print_Pow(self, e):
        b, x = e.base, e.exp
        if x.is_Integer and 1 <= int(x) <= 16:
            return "(" + "*".join([self.parenthesize(b, 100)] * int(x)) + ")"
        if x.is_Integer and -16 <= int(x) <= -1:
            return "(1.0/(" + "*".join([self.parenthesize(b, 100)] * -int(x)) + "))"
        if b.is_Integer and x == sp.Rational(1, 2):  # square roots of the basis constants as literals
            return repr(float(sp.sqrt(b).evalf(30)))
        if b.is_Integer and x == sp.Rational(-1, 2):
            return repr(float((1 / sp.sqrt(b)).evalf(30)))
        return super()._print_Pow(e)

    def _print_Float(self, e):
        return repr(float(e))

    def _print_Rational(self, e):
        return "(%d.0/%d.0)" % (e.p, e.q)

    def _print_Integer(self, e):
        return "%d.0" % int(e)


def _emit(name, args, outs, exprs, symbols_in):
    """One __device__ function accumulating `exprs` into the output arrays named in `outs`."""
    pr = _Printer()
    exprs = [sp.expand(e.subs(RN, 1 / RI)) for e in exprs]
    exprs = [sp.collect(e, symbols_in) for e in exprs]
    rep, red = sp.cse(exprs, symbols=sp.numbered_symbols("c"), optimizations="basic")
    lines = ["__device__ __forceinline__ void %s(%s) {" % (name, args)]
    for sym, val in rep:
        lines.append("  const double %s = %s;" % (sym, pr.doprint(val)))
    for (arr, k), e in zip(outs, red):
        lines.append("  %s[%d] += %s;" % (arr, k, pr.doprint(e)))
    lines.append("}")
    nops = sum(sp.count_ops(v) for _, v in rep) + sum(sp.count_ops(e) for e in red)
    return "\n".join(lines), nops


def generate():
    Hm = blake_image()
    f = sp.symbols("f0:3")
    t = sp.symbols("t0:3")
    s = sp.symbols("s0:5")
    q = sp.symbols("q0:3")
    geo = "double R1, double R2, double R3, double h, double ri, double a2"
    parts = []
    e_s = strain5(source_flows(Hm, None, None, s, None))
    parts.append(_emit("wall_strain_s", geo + ", const double* s, double* e", [("e", c) for c in range(5)],
                       e_s, list(s)))
    e_f = strain5(source_flows(Hm, f, t, None, q))
    parts.append(_emit("wall_strain_ftq", geo + ", const double* f, const double* t, const double* q, double* e",
                       [("e", c) for c in range(5)], e_f, list(f) + list(t) + list(q)))
    U, W = motion(source_flows(Hm, f, t, s, q))
    parts.append(_emit("wall_motion_ftsq", geo + ", const double* f, const double* t, const double* s, "
                       "const double* q, double* u, double* w", [("u", c) for c in range(3)] +
                       [("w", c) for c in range(3)], U + W, list(f) + list(t) + list(s) + list(q)))
    uf = source_flows(Hm, f, t, s, q)
    parts.append(_emit("wall_flow_ftsq", geo + ", const double* f, const double* t, const double* s, "
                       "const double* q, double* u", [("u", c) for c in range(3)], uf,
                       list(f) + list(t) + list(s) + list(q)))
    sym_map = {}
    for sym in list(f) + list(t) + list(s) + list(q):
        nm = str(sym)
        sym_map[nm] = "%s[%s]" % (nm[0], nm[1:])
    body = []
    counts = []
    for (code, nops), nm in zip(parts, ("wall_strain_s", "wall_strain_ftq", "wall_motion_ftsq", "wall_flow_ftsq")):
        for k, v in sym_map.items():
            code = _replace_symbol(code, k, v)
        body.append(code)
        counts.append("//   %-18s %d operations" % (nm, nops))
    head = [
        "// Generated by paper_1411_0278_amd/wall_codegen.py (do not edit): the image-part arithmetic of a",
        "// plane no-slip wall per (receiver, source) pair, from Blake's image system written through 1/R and",
        "// |R| (R = receiver centre or field point minus the source's mirror point, h the source's height",
        "// above the wall, ri = 1/|R|, a2 = a^2; source coefficients pre-scaled: f = P F, t = P T,",
        "// s = P Sigma (5-basis), q = (a^5/20) d, P = 1/(8 pi eta)). Operation counts after sharing:",
    ] + counts + ["#pragma once", "", "namespace mbs {", ""]
    return "\n".join(head) + "\n" + "\n\n".join(body) + "\n\n}  // namespace mbs\n"


def _replace_symbol(code, name, repl):
    import re
    return re.sub(r"\b%s\b" % re.escape(name), repl, code)


def main(argv=None):
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "mbs_wall_gen.h")
    text = generate()
    if argv and "--check" in argv:
        sys.exit(0 if open(out).read() == text else 1)
    with open(out, "w") as fh:
        fh.write(text)
    print("wrote", out)


if __name__ == "__main__":
    main(sys.argv[1:])
