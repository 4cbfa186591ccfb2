"""Independent 50-digit evaluation of the discrete plasma response (mpmath).

A second, deliberately naive implementation of the discrete method for tiny
problems (a few cells, one or two particles per cell, a few slices), written
in plain Python with mpmath at 50 significant digits.  It shares no code with
the C oracle and exists only to pin the oracle's arithmetic: index handling,
operation order and every term of the field equations (WAKE paper,
arXiv:1411.3246, Section II A, Eqs. (1)-(7)).
"""
from __future__ import annotations

import mpmath as mp

mp.mp.dps = 50


def _m(v):
    return mp.mpf(v)


class Grid:
    def __init__(self, p):
        self.p = p
        self.N = p.n_r
        self.h = _m(p.r_max) / p.n_r
        self.cyl = p.geom == "cyl"
        self.dxi = (_m(p.xi_max) - _m(p.xi_min)) / p.n_xi
        self.r = [j * self.h for j in range(self.N + 1)]
        self.V = []
        for j in range(self.N + 1):
            if self.cyl:
                if j == 0:
                    v = mp.pi * self.h ** 2 / 3
                elif j == self.N:
                    v = mp.pi * self.h ** 2 * (self.N - _m(1) / 3)
                else:
                    v = 2 * mp.pi * j * self.h ** 2
            else:
                v = self.h / 2 if j in (0, self.N) else self.h
            self.V.append(v)

    def weights(self, rho):
        u = rho / self.h
        j = int(mp.floor(u))
        j = min(max(j, 0), self.N - 1)
        t = u - j
        return j, t

    def pw(self, r):
        """r^alpha."""
        return r if self.cyl else _m(1)


def load(p, eps):
    g = Grid(p)
    warm = p.u_th > 0
    npos = p.ppc // 2 if warm else p.ppc
    parts = []
    nion = [_m(0)] * (g.N + 1)
    for c in range(g.N):
        for m in range(npos):
            lo = (c + _m(m) / npos) * g.h
            hi = (c + _m(m + 1) / npos) * g.h
            r0 = (c + (m + _m(1) / 2) / npos) * g.h
            area = _m(p.n0) * (mp.pi * (hi * hi - lo * lo) if g.cyl else (hi - lo))
            j, t = g.weights(r0)
            nion[j] += area * (1 - t)
            nion[j + 1] += area * t
            if not warm:
                parts.append(dict(x=r0, y=_m(0), px=_m(0), py=_m(0), d0=_m(1), w=area))
                continue
            q = c * npos + m
            pr, pt, pz = (_m(p.u_th) * _m(float(eps[q][k])) for k in range(3))
            g0 = mp.sqrt(1 + pr * pr + pt * pt + pz * pz)
            for s in (1, -1):
                d0 = g0 - s * pz
                parts.append(dict(x=r0, y=_m(0), px=s * pr, py=s * pt, d0=d0,
                                  w=area / 2 * d0 / g0))
    nion = [nion[j] / g.V[j] for j in range(g.N + 1)]
    return g, parts, nion


def _radial(g, q):
    """(rho, wall sign, parity sign, unfolded r, physical p_r, l^2)."""
    x, y, px, py = q["x"], q["y"], q["px"], q["py"]
    r = mp.sqrt(x * x + y * y) if g.cyl else abs(x)
    sw = _m(1)
    rho = r
    rmax = _m(g.p.r_max)
    if r > rmax:
        sw = _m(-1)
        rho = max(2 * rmax - r, _m(0))
    if g.cyl:
        sg = sw
        pr = sw * (x * px + y * py) / r if r > 0 else _m(0)
        l2 = (x * py - y * px) ** 2
    else:
        sg = (_m(-1) if x < 0 else _m(1)) * sw
        pr = sg * px
        l2 = _m(0)
    return rho, sw, sg, r, pr, l2


def _tridiag(a, b, c, d):
    """Dense Gaussian elimination of the tridiagonal system (no pivoting
    shortcuts beyond the band)."""
    n = len(d)
    A = mp.matrix(n, n)
    for i in range(n):
        A[i, i] = b[i]
        if i > 0:
            A[i, i - 1] = a[i]
        if i < n - 1:
            A[i, i + 1] = c[i]
    x = mp.lu_solve(A, mp.matrix(d))
    return [x[i] for i in range(n)]


def evaluate(g, parts, nion, jb_row):
    N, h = g.N, g.h
    p = g.p
    dep = lambda row, rho, v: _dep(g, row, rho, v)
    S = [_m(0)] * (N + 1)
    for q in parts:
        rho = _radial(g, q)[0]
        dep(S, rho, q["w"])
    S = [S[j] / g.V[j] for j in range(N + 1)]
    # psi
    a, b, c, d = [], [], [], []
    k0 = (2 + (2 if g.cyl else 0)) / h ** 2
    a.append(_m(0)); b.append(-k0); c.append(k0); d.append(S[0] - nion[0])
    for j in range(1, N):
        rj, rm, rp = g.pw(g.r[j]), g.pw(g.r[j] - h / 2), g.pw(g.r[j] + h / 2)
        a.append(rm / (rj * h * h)); c.append(rp / (rj * h * h))
        b.append(-(rm + rp) / (rj * h * h)); d.append(S[j] - nion[j])
    psi = _tridiag(a, b, c, d) + [_m(0)]
    dpsi = [_m(0)] + [(psi[j + 1] - psi[j - 1]) / (2 * h) for j in range(1, N)] + \
           [(psi[N] - psi[N - 1]) / h]
    rows = {k: [_m(0)] * (N + 1) for k in ("Jr", "Jz", "M1", "M2", "M3", "M4", "M5")}
    aux = []
    for q in parts:
        rho, sw, sg, r, pr, l2 = _radial(g, q)
        j, t = g.weights(rho)
        D = q["d0"] + (1 - t) * psi[j] + t * psi[j + 1]
        if D < _m(p.d_min):
            D = _m(p.d_min)
        p2 = q["px"] ** 2 + q["py"] ** 2
        gam = (1 + p2 + D * D) / (2 * D)
        pz = (1 + p2 - D * D) / (2 * D)
        w = q["w"]
        dep(rows["Jr"], rho, -w * pr / D)
        dep(rows["Jz"], rho, -w * pz / D)
        dep(rows["M1"], rho, w / D)
        dep(rows["M2"], rho, w * (gam / D ** 2 - pr * pr / D ** 3))
        if g.cyl and rho > 0:
            dep(rows["M3"], rho, w * l2 / (D ** 2 * rho ** 3))
        dep(rows["M4"], rho, w * pr / D ** 2)
        dep(rows["M5"], rho, w * pr * pr / D ** 2)
        aux.append((D, gam))
    for k in rows:
        rows[k] = [rows[k][j] / g.V[j] for j in range(N + 1)]
    Jz = [rows["Jz"][j] + _m(float(jb_row[j])) for j in range(N + 1)]
    Jr = rows["Jr"]
    Ez = [_m(0)] * (N + 1)
    for j in range(N - 1, -1, -1):
        Ez[j] = Ez[j + 1] - h / 2 * (Jr[j] + Jr[j + 1])
    al = 1 if g.cyl else 0
    a, b, c, d = [], [], [], []
    for j in range(1, N):
        rj = g.r[j]
        a.append(1 / h ** 2 - al / (2 * rj * h))
        b.append(-2 / h ** 2 - al / rj ** 2 - rows["M1"][j])
        c.append(1 / h ** 2 + al / (2 * rj * h))
        d.append((Jz[j + 1] - Jz[j - 1]) / (2 * h) - rows["M2"][j] * dpsi[j]
                 - al * rows["M3"][j] + rows["M4"][j] * Ez[j]
                 + (g.pw(g.r[j + 1]) * rows["M5"][j + 1] - g.pw(g.r[j - 1]) * rows["M5"][j - 1])
                 / (2 * h * g.pw(rj)))
    rh = g.pw(g.r[N] - h / 2)
    a.append(-g.pw(g.r[N - 1]) / (h * rh)); b.append(g.pw(g.r[N]) / (h * rh)); c.append(_m(0))
    d.append((Jz[N] + Jz[N - 1]) / 2)
    B = [_m(0)] + _tridiag(a, b, c, d)
    derivs = []
    for q, (D, gam) in zip(parts, aux):
        rho, sw, sg, r, pr, l2 = _radial(g, q)
        j, t = g.weights(rho)
        F = gam / D * ((1 - t) * dpsi[j] + t * dpsi[j + 1]) - ((1 - t) * B[j] + t * B[j + 1])
        if g.cyl:
            if r > 0:
                derivs.append((q["px"] / D, q["py"] / D, sw * F * q["x"] / r, sw * F * q["y"] / r))
            else:
                derivs.append((q["px"] / D, q["py"] / D, _m(0), _m(0)))
        else:
            derivs.append((q["px"] / D, _m(0), sg * F, _m(0)))
    fields = (psi, Ez, B, [-v for v in dpsi])
    return fields, derivs


def _dep(g, row, rho, v):
    j, t = g.weights(rho)
    row[j] += v * (1 - t)
    row[j + 1] += v * t


def march(p, eps, jb):
    """All stored fields [slice][field][node] of the Heun march."""
    g, parts, nion = load(p, eps)
    out = []
    keys = ("x", "y", "px", "py")
    rmax = _m(p.r_max)
    for k in range(p.n_xi):
        fields, f0 = evaluate(g, parts, nion, jb[k])
        out.append(fields)
        if k == p.n_xi - 1:
            break
        pred = []
        for q, f in zip(parts, f0):
            pq = dict(q)
            for key, fv in zip(keys, f):
                pq[key] = q[key] + g.dxi * fv
            pred.append(pq)
        _, f1 = evaluate(g, pred, nion, jb[k + 1])
        for q, fa, fb in zip(parts, f0, f1):
            for key, va, vb in zip(keys, fa, fb):
                q[key] = q[key] + g.dxi / 2 * (va + vb)
            # outer wall
            if g.cyl:
                r = mp.sqrt(q["x"] ** 2 + q["y"] ** 2)
                if r > rmax:
                    rn = max(2 * rmax - r, _m(0))
                    ux, uy = q["x"] / r, q["y"] / r
                    prr = ux * q["px"] + uy * q["py"]
                    q["x"], q["y"] = rn * ux, rn * uy
                    q["px"] -= 2 * prr * ux
                    q["py"] -= 2 * prr * uy
            else:
                if abs(q["x"]) > rmax:
                    xn = max(2 * rmax - abs(q["x"]), _m(0))
                    q["x"] = -xn if q["x"] < 0 else xn
                    q["px"] = -q["px"]
    return out, parts
