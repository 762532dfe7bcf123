"""Writes csrc/mbs_periodic_gen.h: the per-pair and per-wave-vector arithmetic of spheres in a
periodic cubic box (Ewald summation of the periodic Oseen tensor).

Run from the repository root after changing the derivation (the header is committed; the library
build only compiles it):

    python -m paper_1411_0278_amd.periodic_codegen            (--check: compare only, exit status 1 if
                                                                the committed header differs)

The periodic Oseen tensor with zero mean velocity over the box (Hasimoto's procedure) is split with
a parameter xi into a real-space part summed over the images within a cutoff and a Fourier part
summed over the reciprocal lattice. Since G = (delta lap - grad grad) |x|, the parts are written
through one scalar each:

    real space:     G^R = (delta lap - grad grad) B(r),   B(r) = r erfc(xi r) - exp(-xi^2 r^2) / (xi sqrt(pi))
    Fourier space:  G^(k) = (delta k^2 - k k) 8 pi / k^4 (1 + k^2/(4 xi^2)) exp(-k^2/(4 xi^2))

(the transform of B is -8 pi / k^4 times one minus the splitting factor). Each Galerkin block is the
free-space operator chain applied to the part: the source's flow (force F^0 G f, torque
(1/2) curl (G t), stresslet F^1 d_k G_ij s_jk, rank-3 mode -lap G q) and the receiver's projection
(U = F^0 u, W = (1/2) curl u, E = sym grad F^1 u, 5-basis), F^l = 1 + a^2/(4l+6) lap. Per unit of
the pre-scaled source coefficients f = P F, t = P T, s = P Sigma (5-basis), q = (a^5/20) d,
P = 1/(8 pi eta):

    real space (x the separation, r = |x|, ri = 1/r, ec = erfc(xi r), ex = exp(-xi^2 r^2)):
        per_real_strain_s, per_real_strain_ftq, per_real_motion_ftsq   (accumulate e[5] / u[3], w[3]),
        per_real_flow_ftsq (the flow itself at a field point, accumulate u[3]),
        per_real_es_radial (the radial functions al, be, ga of the stresslet strain's isotropic form
        E = al Sigma + be (x (Sigma x) + (Sigma x) x) + ga (x.Sigma x) x x + (trace), which the operator
        pass contracts itself: about a tenth of the operations of per_real_strain_s),
        per_real_ftq_radial (the five radial functions of the strain of a force, a torque and the
        rank-3 mode, E = x a + a x + b x x, a = Af f + Aq q + Dt (x cross t), b = Bf (x.f) + Bq (x.q)),
        per_real_motion_radial (the twelve of the rigid-body motion, U = F1 f + Q1 q + S1 w + T1 (t cross x)
        + (F2 (x.f) + Q2 (x.q) + S2 (x.w)) x, W = G1 (f cross x) + Gq (q cross x) + J1 (x cross w) + H1 t
        + H2 (x.t) x, w = Sigma x), contracted by the right-hand side and output passes,
        per_real_flow_radial (the seven of the flow at a field point, the U form without the receiver's
        operator), contracted by the flow pass
    Fourier space (k, ik2 = 1/k^2, the complex structure factors of the coefficients split into real
    and imaginary parts; the splitting factor and 1/L^3 applied by the caller):
        per_hat_strain_s, per_hat_strain_ftq, per_hat_motion_ftsq, per_hat_flow_ftsq
                                                                       (write the complex targets)
    a sphere's smooth part at its own centre, (1/(2 pi)^3) integral of the multiplier over all k
    (isotropic: a multiple of the identity for the blocks that do not vanish by parity):
        per_self_es, per_self_uf, per_self_ud, per_self_wt

The real-space polynomials are reduced with x^2 = r^2 - y^2 - z^2 and grouped by source coefficient;
common subexpressions are shared within each function.
"""
from __future__ import annotations

import os
import re
import sys

import sympy as sp
from sympy.printing.c import C99CodePrinter

X1, X2, X3 = sp.symbols("x1 x2 x3", real=True)
RR, XI, A2 = sp.symbols("rr xi a2", positive=True)
EC, EX = sp.symbols("ec ex", positive=True)
RI = sp.symbols("ri", positive=True)
K1, K2, K3 = sp.symbols("k1 k2 k3", real=True)
IK2 = sp.symbols("ik2", positive=True)
_XV, _KV = (X1, X2, X3), (K1, K2, K3)
_S2, _S6 = 1 / sp.sqrt(2), 1 / sp.sqrt(6)
_B5 = (
    ((_S2, 0, 0), (0, -_S2, 0), (0, 0, 0)),
    ((-_S6, 0, 0), (0, -_S6, 0), (0, 0, 2 * _S6)),
    ((0, _S2, 0), (_S2, 0, 0), (0, 0, 0)),
    ((0, 0, _S2), (0, 0, 0), (_S2, 0, 0)),
    ((0, 0, 0), (0, 0, _S2), (0, _S2, 0)),
)


# ------------------------------------------------------------------ two representations
class _Real:
    """Functions of x1..x3, rr, ec, ex: d/dx_i through x_i and through rr (drr/dx_i = x_i / rr),
    d ec/drr = -(2 xi/sqrt(pi)) ex, d ex/drr = -2 xi^2 rr ex."""

    @staticmethod
    def red(f):
        f = sp.expand(f)
        f = f.replace(lambda e: e.is_Pow and e.base == X1 and e.exp.is_Integer and e.exp >= 2,
                      lambda e: X1 ** (int(e.exp) % 2) * (RR ** 2 - X2 ** 2 - X3 ** 2) ** (int(e.exp) // 2))
        return sp.expand(f)

    def d(self, f, i):
        dr = sp.diff(f, RR) - 2 * XI / sp.sqrt(sp.pi) * EX * sp.diff(f, EC) - 2 * XI ** 2 * RR * EX * sp.diff(f, EX)
        return self.red(sp.diff(f, _XV[i]) + _XV[i] / RR * dr)

    def lap(self, f):
        return self.red(sum(self.d(self.d(f, i), i) for i in range(3)))

    def kernel(self):
        b = RR * EC - EX / (XI * sp.sqrt(sp.pi))
        lb = self.lap(b)
        return [[self.red(int(i == j) * lb - self.d(self.d(b, i), j)) for j in range(3)] for i in range(3)]


class _Fourier:
    """Functions of k1..k3 and ik2 = 1/k^2: d/dx_i -> i k_i, lap -> -k^2."""

    @staticmethod
    def red(f):
        f = sp.expand(f)
        k2 = K1 ** 2 + K2 ** 2 + K3 ** 2
        # k^2 ik2 = 1 on every monomial (k1^2 replaced by 1/ik2 - k2^2 - k3^2 repeatedly)
        f = f.replace(lambda e: e.is_Pow and e.base == K1 and e.exp.is_Integer and e.exp >= 2,
                      lambda e: K1 ** (int(e.exp) % 2) * (1 / IK2 - K2 ** 2 - K3 ** 2) ** (int(e.exp) // 2))
        return sp.expand(f)

    def d(self, f, i):
        return self.red(sp.I * _KV[i] * f)

    def lap(self, f):
        return self.red(-f / IK2)

    def kernel(self):
        return [[self.red((int(i == j) / IK2 - _KV[i] * _KV[j]) * 8 * sp.pi * IK2 ** 2) for j in range(3)]
                for i in range(3)]


def _faxen(rep, f, l):
    return rep.red(f + A2 / (4 * l + 6) * rep.lap(f))


def source_flow(rep, K, f, t, s, q):
    """u_i of the pre-scaled coefficients (any may be None)."""
    u = [0, 0, 0]
    for i in range(3):
        acc = 0
        if f is not None:
            acc += _faxen(rep, sum(K[i][j] * f[j] for j in range(3)), 0)
        if s is not None:
            Sc = [[sum(s[c] * _B5[c][j][k] for c in range(5)) for k in range(3)] for j in range(3)]
            acc += _faxen(rep, sum(rep.d(K[i][j], k) * Sc[j][k] for j in range(3) for k in range(3) if Sc[j][k] != 0), 1)
        if q is not None:
            acc += -sum(rep.lap(K[i][j]) * q[j] for j in range(3))
        u[i] = acc
    if t is not None:  # (1/2) curl of G t
        g = [sum(K[i][j] * t[j] for j in range(3)) for i in range(3)]
        for i in range(3):
            u[i] += sp.Rational(1, 2) * (rep.d(g[(i + 2) % 3], (i + 1) % 3) - rep.d(g[(i + 1) % 3], (i + 2) % 3))
    return [rep.red(ui) for ui in u]


def strain5(rep, u):
    v = [_faxen(rep, ui, 1) for ui in u]
    return [rep.red(sum(_B5[c][i][j] * sp.Rational(1, 2) * (rep.d(v[i], j) + rep.d(v[j], i))
                        for i in range(3) for j in range(3) if _B5[c][i][j] != 0)) for c in range(5)]


def motion(rep, u):
    U = [_faxen(rep, ui, 0) for ui in u]
    W = [rep.red(sp.Rational(1, 2) * (rep.d(u[(i + 2) % 3], (i + 1) % 3) - rep.d(u[(i + 1) % 3], (i + 2) % 3)))
         for i in range(3)]
    return U, W


# ------------------------------------------------------------------ the self constants
def _sphere_average(mono_exps):
    """Average over the unit sphere of n1^a n2^b n3^c: (a-1)!!(b-1)!!(c-1)!!/(a+b+c+1)!! for even
    exponents, 0 otherwise."""
    a, b, c = mono_exps
    if a % 2 or b % 2 or c % 2:
        return sp.Integer(0)
    df = lambda m: sp.factorial2(m - 1) if m > 0 else sp.Integer(1)  # noqa: E731
    return df(a) * df(b) * df(c) / sp.factorial2(a + b + c + 1)


def self_constant(expr):
    """(1/(2 pi)^3) integral over k-space of expr(k) times the splitting factor, exactly: the
    multiplier is a sum of monomials k1^a k2^b k3^c ik2^m, each the sphere average of the direction
    times a radial Gaussian moment."""
    kk = sp.symbols("kk", positive=True)
    total = 0
    for term in sp.Add.make_args(sp.expand(expr)):
        pw = term.as_powers_dict()
        a, b, c, m = (int(pw.get(v, 0)) for v in (K1, K2, K3, IK2))
        coef = term / (K1 ** a * K2 ** b * K3 ** c * IK2 ** m)
        ang = _sphere_average((a, b, c))
        if ang == 0:
            continue
        deg = a + b + c - 2 * m  # the radial power of the monomial
        radial = sp.integrate(kk ** (deg + 2) * (1 + kk ** 2 / (4 * XI ** 2)) * sp.exp(-kk ** 2 / (4 * XI ** 2)),
                              (kk, 0, sp.oo))
        total += sp.simplify(coef) * ang * 4 * sp.pi * radial
    return sp.simplify(total / (2 * sp.pi) ** 3)


# ------------------------------------------------------------------ printing
class _Printer(C99CodePrinter):
    def _print_Pow(self, e):
        b, x = e.base, e.exp
        if x.is_Integer and 1 <= int(x) <= 16:
            return "(" + "*".join([self.parenthesize(b, 100)] * int(x)) + ")"
        if x.is_Integer and -16 <= int(x) <= -1:
            return "(1.0/(" + "*".join([self.parenthesize(b, 100)] * -int(x)) + "))"
        if b.is_Number and (x == sp.Rational(1, 2) or x == sp.Rational(-1, 2)):
            return repr(float(sp.N(e, 30)))
        return super()._print_Pow(e)

    def _print_Float(self, e):
        return repr(float(e))

    def _print_Rational(self, e):
        return "(%d.0/%d.0)" % (e.p, e.q)

    def _print_Integer(self, e):
        return "%d.0" % int(e)

    def _print_Pi(self, e):
        return repr(float(sp.pi.evalf(30)))


def _numeric(e):
    """Exact constants (pi, square roots) to binary64 literals."""
    return e.xreplace({s: sp.Float(sp.N(s, 30), 30) for s in e.atoms(sp.Pow) if s.is_number}).xreplace(
        {sp.pi: sp.Float(sp.N(sp.pi, 30), 30)})


def _emit(name, args, outs, exprs, symbols_in, subs=None):
    pr = _Printer()
    if subs:
        exprs = [sp.expand(e.subs(subs)) for e in exprs]
    exprs = [sp.collect(sp.expand(_numeric(e)), symbols_in) for e in exprs]
    rep, red = sp.cse(exprs, symbols=sp.numbered_symbols("c"), optimizations="basic")
    lines = ["__device__ __forceinline__ void %s(%s) {" % (name, args)]
    for sym, val in rep:
        lines.append("  const double %s = %s;" % (sym, pr.doprint(val)))
    for (arr, k, op), e in zip(outs, red):
        lines.append("  %s[%d] %s %s;" % (arr, k, op, pr.doprint(e)))
    lines.append("}")
    nops = sum(sp.count_ops(v) for _, v in rep) + sum(sp.count_ops(e) for e in red)
    return "\n".join(lines), nops


def _complex_parts(exprs, coeffs, re_syms, im_syms):
    """exprs linear in `coeffs` (complex multipliers); returns the real and imaginary parts of
    sum_c M_c (re_c + i im_c) with the symbols of the k-representation real."""
    out_re, out_im = [], []
    for e in exprs:
        e = sp.expand(e)
        r_acc, i_acc = 0, 0
        for cf, rs, is_ in zip(coeffs, re_syms, im_syms):
            m = sp.expand(e.coeff(cf))
            mr = sp.expand((m + m.subs(sp.I, -sp.I)) / 2)
            mi = sp.expand((m - m.subs(sp.I, -sp.I)) / (2 * sp.I))
            r_acc += mr * rs - mi * is_
            i_acc += mr * is_ + mi * rs
        out_re.append(sp.expand(r_acc))
        out_im.append(sp.expand(i_acc))
    return out_re, out_im


def stresslet_radial():
    """The real-space strain of a stresslet through the screened kernel in its isotropic form,
    E = al Sigma + be (x (Sigma x) + (Sigma x) x) + ga (x.Sigma x) x x + de (x.Sigma x) I: the radial
    functions read off along the z axis and the form then checked for a general separation."""
    rl = _Real()
    K = rl.kernel()
    sxx, syy, sxy, sxz, syz = sp.symbols("sxx syy sxy sxz syz", real=True)
    S = [[sxx, sxy, sxz], [sxy, syy, syz], [sxz, syz, -sxx - syy]]
    u = [_faxen(rl, sum(rl.d(K[i][j], k) * S[j][k] for j in range(3) for k in range(3)), 1) for i in range(3)]
    v = [_faxen(rl, ui, 1) for ui in u]
    E = [[rl.red(sp.Rational(1, 2) * (rl.d(v[i], j) + rl.d(v[j], i))) for j in range(3)] for i in range(3)]
    z = {X1: 0, X2: 0, X3: RR}
    Ez = [[sp.expand(E[i][j].subs(z)) for j in range(3)] for i in range(3)]
    al = sp.expand(Ez[0][1].coeff(sxy))
    be = sp.expand((Ez[0][2].coeff(sxz) - al) / RR ** 2)
    de = sp.expand(-(Ez[0][0] - al * sxx).coeff(syy) / RR ** 2)
    ga = sp.expand((-Ez[2][2].coeff(syy) - al - 2 * be * RR ** 2 - de * RR ** 2) / RR ** 4)
    w = [sum(S[i][j] * _XV[j] for j in range(3)) for i in range(3)]
    q = sum(_XV[i] * w[i] for i in range(3))
    for i in range(3):
        for j in range(i, 3):
            form = al * S[i][j] + be * (_XV[i] * w[j] + w[i] * _XV[j]) + ga * q * _XV[i] * _XV[j] + de * q * int(i == j)
            if rl.red(E[i][j] - form) != 0:
                raise AssertionError("the screened stresslet strain is not of the isotropic form")
    return al, be, ga


def _cart_strain(rl, u):
    """Cartesian strain sym grad F^1 u of a flow (the receiver's Faxen operator applied first)."""
    v = [_faxen(rl, ui, 1) for ui in u]
    return [[rl.red(sp.Rational(1, 2) * (rl.d(v[i], j) + rl.d(v[j], i))) for j in range(3)] for i in range(3)]


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _check_form(rl, exact, form, what):
    for e, g in zip(exact, form):
        if rl.red(e - g) != 0:
            raise AssertionError("the screened %s is not of the isotropic form" % what)


def rhs_radial():
    """The real-space strain of a force, a torque and the rank-3 trace mode through the screened
    kernel in isotropic form: E = x a + a x + b x x (+ a trace the 5-basis drops) with
    a = Af f + Aq q + Dt (x cross t) and b = Bf (x.f) + Bq (x.q); the five radial functions read off along the z axis
    and the form checked for a general separation."""
    rl = _Real()
    K = rl.kernel()
    f = sp.symbols("f0:3", real=True)
    t = sp.symbols("t0:3", real=True)
    q = sp.symbols("q0:3", real=True)
    z = {X1: 0, X2: 0, X3: RR}
    out = {}
    for name, vec in (("f", f), ("q", q)):
        E = _cart_strain(rl, source_flow(rl, K, f if name == "f" else None, None, None, q if name == "q" else None))
        Ez = [[sp.expand(E[i][j].subs(z)) for j in range(3)] for i in range(3)]
        A = sp.expand(Ez[0][2].coeff(vec[0]) / RR)
        C = sp.expand(Ez[0][0].coeff(vec[2]) / RR)
        B = sp.expand((Ez[2][2].coeff(vec[2]) - 2 * A * RR - C * RR) / RR ** 3)
        xv = sum(_XV[i] * vec[i] for i in range(3))
        _check_form(rl, [E[i][j] for i in range(3) for j in range(i, 3)],
                    [A * (_XV[i] * vec[j] + vec[i] * _XV[j]) + B * xv * _XV[i] * _XV[j] + C * xv * int(i == j)
                     for i in range(3) for j in range(i, 3)], "strain of a vector source")
        out["A" + name], out["B" + name] = A, B
    E = _cart_strain(rl, source_flow(rl, K, None, t, None, None))
    Ez = [[sp.expand(E[i][j].subs(z)) for j in range(3)] for i in range(3)]
    D = sp.expand(-Ez[0][2].coeff(t[1]) / RR ** 2)
    xt = _cross(_XV, t)
    _check_form(rl, [E[i][j] for i in range(3) for j in range(i, 3)],
                [D * (xt[i] * _XV[j] + _XV[i] * xt[j]) for i in range(3) for j in range(i, 3)], "strain of a torque")
    return [out["Af"], out["Bf"], out["Aq"], out["Bq"], D]


def motion_radial():
    """The real-space rigid-body motion of a sphere (U = F^0 u, W = (1/2) curl u) driven by a force,
    a torque, a stresslet and the rank-3 trace mode through the screened kernel in isotropic form:
        U = F1 f + Q1 q + S1 w + T1 (t cross x) + (F2 (x.f) + Q2 (x.q) + S2 (x.w)) x,   w = Sigma x,
        W = G1 (f cross x) + Gq (q cross x) + J1 (x cross w) + H1 t + H2 (x.t) x;
    the twelve radial functions [F1, F2, Q1, Q2, T1, S1, S2, G1, Gq, H1, H2, J1] read off along the z
    axis and the forms checked for a general separation."""
    rl = _Real()
    K = rl.kernel()
    f = sp.symbols("f0:3", real=True)
    t = sp.symbols("t0:3", real=True)
    q = sp.symbols("q0:3", real=True)
    sxx, syy, sxy, sxz, syz = sp.symbols("sxx syy sxy sxz syz", real=True)
    S = [[sxx, sxy, sxz], [sxy, syy, syz], [sxz, syz, -sxx - syy]]
    # the stresslet through Cartesian components (the 5-basis maps onto them linearly)
    uS = [_faxen(rl, sum(rl.d(K[i][j], k) * S[j][k] for j in range(3) for k in range(3)), 1) for i in range(3)]
    z = {X1: 0, X2: 0, X3: RR}
    r = {}
    for name, vec in (("F", f), ("Q", q)):
        U, W = motion(rl, source_flow(rl, K, f if name == "F" else None, None, None, q if name == "Q" else None))
        Uz = [sp.expand(c.subs(z)) for c in U]
        Wz = [sp.expand(c.subs(z)) for c in W]
        c1 = sp.expand(Uz[0].coeff(vec[0]))
        c2 = sp.expand((Uz[2].coeff(vec[2]) - c1) / RR ** 2)
        g = sp.expand(Wz[0].coeff(vec[1]) / RR)  # W = g (v cross x): along z, W_x = g r v_y
        xv = sum(_XV[i] * vec[i] for i in range(3))
        vx = _cross(vec, _XV)
        _check_form(rl, U, [c1 * vec[i] + c2 * xv * _XV[i] for i in range(3)], "motion of a vector source")
        _check_form(rl, W, [g * vx[i] for i in range(3)], "rotation of a vector source")
        r[name + "1"], r[name + "2"], r["G" + name] = c1, c2, g
    U, W = motion(rl, source_flow(rl, K, None, t, None, None))
    Uz = [sp.expand(c.subs(z)) for c in U]
    Wz = [sp.expand(c.subs(z)) for c in W]
    T1 = sp.expand(Uz[0].coeff(t[1]) / RR)
    H1 = sp.expand(Wz[0].coeff(t[0]))
    H2 = sp.expand((Wz[2].coeff(t[2]) - H1) / RR ** 2)
    tx = _cross(t, _XV)
    xt = sum(_XV[i] * t[i] for i in range(3))
    _check_form(rl, U, [T1 * tx[i] for i in range(3)], "motion of a torque")
    _check_form(rl, W, [H1 * t[i] + H2 * xt * _XV[i] for i in range(3)], "rotation of a torque")
    U = [_faxen(rl, ui, 0) for ui in uS]
    W = [rl.red(sp.Rational(1, 2) * (rl.d(uS[(i + 2) % 3], (i + 1) % 3) - rl.d(uS[(i + 1) % 3], (i + 2) % 3)))
         for i in range(3)]
    Uz = [sp.expand(c.subs(z)) for c in U]
    Wz = [sp.expand(c.subs(z)) for c in W]
    S1 = sp.expand(Uz[0].coeff(sxz) / RR)
    S2 = sp.expand((-Uz[2].coeff(sxx) - S1 * RR) / RR ** 3)  # S_zz = -sxx - syy
    J1 = sp.expand(-Wz[0].coeff(syz) / RR ** 2)
    w = [sum(S[i][j] * _XV[j] for j in range(3)) for i in range(3)]
    xw = sum(_XV[i] * w[i] for i in range(3))
    xcw = _cross(_XV, w)
    _check_form(rl, U, [S1 * w[i] + S2 * xw * _XV[i] for i in range(3)], "motion of a stresslet")
    _check_form(rl, W, [J1 * xcw[i] for i in range(3)], "rotation of a stresslet")
    return [r["F1"], r["F2"], r["Q1"], r["Q2"], T1, S1, S2, r["GF"], r["GQ"], H1, H2, J1]


def flow_radial():
    """The real-space flow itself at a field point (no receiver operator) of a force, a torque, a
    stresslet and the rank-3 trace mode through the screened kernel in isotropic form,
        u = F1 f + Q1 q + S1 w + T1 (t cross x) + (F2 (x.f) + Q2 (x.q) + S2 (x.w)) x,   w = Sigma x;
    the seven radial functions [F1, F2, Q1, Q2, T1, S1, S2] read off along the z axis and the form
    checked for a general separation."""
    rl = _Real()
    K = rl.kernel()
    f = sp.symbols("f0:3", real=True)
    t = sp.symbols("t0:3", real=True)
    q = sp.symbols("q0:3", real=True)
    sxx, syy, sxy, sxz, syz = sp.symbols("sxx syy sxy sxz syz", real=True)
    S = [[sxx, sxy, sxz], [sxy, syy, syz], [sxz, syz, -sxx - syy]]
    z = {X1: 0, X2: 0, X3: RR}
    r = {}
    for name, vec in (("F", f), ("Q", q)):
        u = source_flow(rl, K, f if name == "F" else None, None, None, q if name == "Q" else None)
        uz = [sp.expand(c.subs(z)) for c in u]
        c1 = sp.expand(uz[0].coeff(vec[0]))
        c2 = sp.expand((uz[2].coeff(vec[2]) - c1) / RR ** 2)
        xv = sum(_XV[i] * vec[i] for i in range(3))
        _check_form(rl, u, [c1 * vec[i] + c2 * xv * _XV[i] for i in range(3)], "flow of a vector source")
        r[name + "1"], r[name + "2"] = c1, c2
    u = source_flow(rl, K, None, t, None, None)
    uz = [sp.expand(c.subs(z)) for c in u]
    T1 = sp.expand(uz[0].coeff(t[1]) / RR)
    tx = _cross(t, _XV)
    _check_form(rl, u, [T1 * tx[i] for i in range(3)], "flow of a torque")
    u = [_faxen(rl, sum(rl.d(K[i][j], k) * S[j][k] for j in range(3) for k in range(3)), 1) for i in range(3)]
    uz = [sp.expand(c.subs(z)) for c in u]
    S1 = sp.expand(uz[0].coeff(sxz) / RR)
    S2 = sp.expand((-uz[2].coeff(sxx) - S1 * RR) / RR ** 3)
    w = [sum(S[i][j] * _XV[j] for j in range(3)) for i in range(3)]
    xw = sum(_XV[i] * w[i] for i in range(3))
    _check_form(rl, u, [S1 * w[i] + S2 * xw * _XV[i] for i in range(3)], "flow of a stresslet")
    return [r["F1"], r["F2"], r["Q1"], r["Q2"], T1, S1, S2]


def generate():
    f = sp.symbols("f0:3")
    t = sp.symbols("t0:3")
    s = sp.symbols("s0:5")
    q = sp.symbols("q0:3")
    parts = []
    # real space
    rl = _Real()
    Kr = rl.kernel()
    geo = "double x1, double x2, double x3, double ri, double ec, double ex, double xi, double a2"
    sub = {RR: 1 / RI}
    e_s = strain5(rl, source_flow(rl, Kr, None, None, s, None))
    parts.append(_emit("per_real_strain_s", geo + ", const double* s, double* e", [("e", c, "+=") for c in range(5)],
                       e_s, list(s), sub))
    e_f = strain5(rl, source_flow(rl, Kr, f, t, None, q))
    parts.append(_emit("per_real_strain_ftq", geo + ", const double* f, const double* t, const double* q, double* e",
                       [("e", c, "+=") for c in range(5)], e_f, list(f) + list(t) + list(q), sub))
    U, W = motion(rl, source_flow(rl, Kr, f, t, s, q))
    parts.append(_emit("per_real_motion_ftsq", geo + ", const double* f, const double* t, const double* s, "
                       "const double* q, double* u, double* w", [("u", c, "+=") for c in range(3)] +
                       [("w", c, "+=") for c in range(3)], U + W, list(f) + list(t) + list(s) + list(q), sub))
    al, be, ga = stresslet_radial()
    parts.append(_emit("per_real_es_radial", "double ri, double ec, double ex, double xi, double a2, double* abg",
                       [("abg", 0, "="), ("abg", 1, "="), ("abg", 2, "=")], [al, be, ga], [EC, EX], sub))
    parts.append(_emit("per_real_ftq_radial", "double ri, double ec, double ex, double xi, double a2, double* rf",
                       [("rf", c, "=") for c in range(5)], rhs_radial(), [EC, EX], sub))
    parts.append(_emit("per_real_motion_radial", "double ri, double ec, double ex, double xi, double a2, double* rm",
                       [("rm", c, "=") for c in range(12)], motion_radial(), [EC, EX], sub))
    parts.append(_emit("per_real_flow_radial", "double ri, double ec, double ex, double xi, double a2, double* rw",
                       [("rw", c, "=") for c in range(7)], flow_radial(), [EC, EX], sub))
    ff = source_flow(rl, Kr, f, t, s, q)
    parts.append(_emit("per_real_flow_ftsq", geo + ", const double* f, const double* t, const double* s, "
                       "const double* q, double* u", [("u", c, "+=") for c in range(3)], ff,
                       list(f) + list(t) + list(s) + list(q), sub))
    # Fourier space: complex structure factors in, complex targets out
    fo = _Fourier()
    Kf = fo.kernel()
    kgeo = "double k1, double k2, double k3, double ik2, double a2"
    sr, si = sp.symbols("sr0:5"), sp.symbols("si0:5")
    fr, fi = sp.symbols("fr0:3"), sp.symbols("fi0:3")
    tr, ti = sp.symbols("tr0:3"), sp.symbols("ti0:3")
    qr, qi = sp.symbols("qr0:3"), sp.symbols("qi0:3")
    hs = strain5(fo, source_flow(fo, Kf, None, None, s, None))
    re_, im_ = _complex_parts(hs, s, sr, si)
    parts.append(_emit("per_hat_strain_s", kgeo + ", const double* sr, const double* si, double* er, double* ei",
                       [("er", c, "=") for c in range(5)] + [("ei", c, "=") for c in range(5)], re_ + im_,
                       list(sr) + list(si)))
    hf = strain5(fo, source_flow(fo, Kf, f, t, None, q))
    re_, im_ = _complex_parts(hf, list(f) + list(t) + list(q), list(fr) + list(tr) + list(qr), list(fi) + list(ti) + list(qi))
    parts.append(_emit("per_hat_strain_ftq", kgeo + ", const double* fr, const double* fi, const double* tr, "
                       "const double* ti, const double* qr, const double* qi, double* er, double* ei",
                       [("er", c, "=") for c in range(5)] + [("ei", c, "=") for c in range(5)], re_ + im_,
                       list(fr) + list(fi) + list(tr) + list(ti) + list(qr) + list(qi)))
    hU, hW = motion(fo, source_flow(fo, Kf, f, t, s, q))
    re_, im_ = _complex_parts(hU + hW, list(f) + list(t) + list(s) + list(q), list(fr) + list(tr) + list(sr) + list(qr),
                              list(fi) + list(ti) + list(si) + list(qi))
    parts.append(_emit("per_hat_motion_ftsq", kgeo + ", const double* fr, const double* fi, const double* tr, "
                       "const double* ti, const double* sr, const double* si, const double* qr, const double* qi, "
                       "double* ur, double* ui", [("ur", c, "=") for c in range(6)] + [("ui", c, "=") for c in range(6)],
                       re_ + im_, list(fr) + list(fi) + list(tr) + list(ti) + list(sr) + list(si) + list(qr) + list(qi)))
    hf3 = source_flow(fo, Kf, f, t, s, q)
    re_, im_ = _complex_parts(hf3, list(f) + list(t) + list(s) + list(q), list(fr) + list(tr) + list(sr) + list(qr),
                              list(fi) + list(ti) + list(si) + list(qi))
    parts.append(_emit("per_hat_flow_ftsq", kgeo + ", const double* fr, const double* fi, const double* tr, "
                       "const double* ti, const double* sr, const double* si, const double* qr, const double* qi, "
                       "double* ur, double* ui", [("ur", c, "=") for c in range(3)] + [("ui", c, "=") for c in range(3)],
                       re_ + im_, list(fr) + list(fi) + list(tr) + list(ti) + list(sr) + list(si) + list(qr) + list(qi)))
    # self constants: the diagonal of the isotropic blocks, per unit P (E from s, U from f, U from q, W from t)
    consts = {}
    unit = lambda syms, k: [sp.Integer(int(i == k)) for i in range(len(syms))]  # noqa: E731
    es0 = strain5(fo, source_flow(fo, Kf, None, None, unit(s, 0), None))[0]
    consts["per_self_es"] = self_constant(es0)
    Uf, _ = motion(fo, source_flow(fo, Kf, unit(f, 0), None, None, None))
    consts["per_self_uf"] = self_constant(Uf[0])
    Uq, _ = motion(fo, source_flow(fo, Kf, None, None, None, unit(q, 0)))
    consts["per_self_ud"] = self_constant(Uq[0])
    _, Wt = motion(fo, source_flow(fo, Kf, None, unit(t, 0), None, None))
    consts["per_self_wt"] = self_constant(Wt[0])
    pr = _Printer()
    cparts = []
    for nm, val in consts.items():
        v = sp.simplify(val)
        cparts.append("__host__ __device__ inline double %s(double xi, double a2) { return %s; }"
                      % (nm, pr.doprint(_numeric(v))))
    sym_map = {}
    for group in (f, t, s, q, sr, si, fr, fi, tr, ti, qr, qi):
        for sym in group:
            nm = str(sym)
            m = re.match(r"([a-z]+)(\d+)$", nm)
            sym_map[nm] = "%s[%s]" % (m.group(1), m.group(2))
    names = ("per_real_strain_s", "per_real_strain_ftq", "per_real_motion_ftsq", "per_real_es_radial",
             "per_real_ftq_radial", "per_real_motion_radial", "per_real_flow_radial", "per_real_flow_ftsq",
             "per_hat_strain_s", "per_hat_strain_ftq", "per_hat_motion_ftsq", "per_hat_flow_ftsq")
    body, counts = [], []
    for (code, nops), nm in zip(parts, names):
        for k, v in sym_map.items():
            code = re.sub(r"\b%s\b" % re.escape(k), v, code)
        body.append(code)
        counts.append("//   %-22s %d operations" % (nm, nops))
    head = [
        "// Generated by paper_1411_0278_amd/periodic_codegen.py (do not edit): Ewald summation of the",
        "// periodic Oseen tensor for spheres in a cubic box. Real space: x the separation (minimum image),",
        "// ri = 1/|x|, ec = erfc(xi |x|), ex = exp(-xi^2 |x|^2); Fourier space: k, ik2 = 1/k^2, complex",
        "// structure factors in, complex targets out (splitting factor and 1/L^3 applied by the caller).",
        "// Source coefficients pre-scaled: f = P F, t = P T, s = P Sigma (5-basis), q = (a^5/20) d,",
        "// P = 1/(8 pi eta); the self constants are per unit P. Operation counts after sharing:",
    ] + counts + ["#pragma once", "", "namespace mbs {", ""]
    return "\n".join(head) + "\n" + "\n\n".join(body) + "\n\n" + "\n".join(cparts) + "\n\n}  // namespace mbs\n"


def main(argv=None):
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "mbs_periodic_gen.h")
    text = generate()
    if argv and "--check" in argv:  # the committed header is what the derivation writes
        same = open(out).read() == text
        print("up to date" if same else "differs from the derivation", out)
        sys.exit(0 if same else 1)
    with open(out, "w") as fh:
        fh.write(text)
    print("wrote", out)


if __name__ == "__main__":
    main(sys.argv[1:])
