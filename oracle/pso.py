"""Reference constriction PSO and elitist mutation, FP64 (test infrastructure only).

Written from the paper's Theory section: Eq. 1 (velocity update with
constriction factor chi, cognitive c1 and social c2 terms, independent U[0,1]
vectors u1, u2 multiplied element by element), Eq. 2 (position update), Eq. 3
(chi as a function of phi = c1 + c2 >= 4) and the elitist-mutation figure
(the NM worst particles take the global best, each coordinate perturbed with
probability p_em by 0.1 * VR_d * N(0, 1), velocities unchanged). Random draws
are inputs, so the same numbers can drive this and the product driver.

Readings where the paper is silent or inconsistent:
  * "worst" = largest misfit (the search minimises); ties keep index order.
  * velocities are clamped to [-lambda VR, lambda VR] (pso.lambda key) and
    positions to the search box after each move (the paper returns
    out-of-bounds variables to the box without saying how); the velocity is
    kept when a position is clamped.
  * the personal best is replaced only on strict improvement; the global best
    is the lowest personal best, ties to the lowest index.
Pinned by: chi closed forms, hand-worked special cases and invariants (tests).
"""
import math

import numpy as np


def constriction(c1, c2):
    """Eq. 3: chi = 2 / |2 - phi - sqrt(phi^2 - 4 phi)|, phi = c1 + c2 >= 4."""
    phi = c1 + c2
    if phi < 4.0:
        raise ValueError("phi = c1 + c2 must be >= 4")
    return 2.0 / abs(2.0 - phi - math.sqrt(phi * phi - 4.0 * phi))


def update_bests(x, f, p, fp):
    """Personal bests (strict improvement) and the gbest index (ties -> lowest)."""
    N = x.shape[0]
    p = p.copy()
    fp = fp.copy()
    for i in range(N):
        if f[i] < fp[i]:
            fp[i] = f[i]
            p[i, :] = x[i, :]
    gi = 0
    for i in range(1, N):
        if fp[i] < fp[gi]:
            gi = i
    return p, fp, gi


def move(x, v, p, g, u1, u2, chi, c1, c2, vclamp, lo, hi):
    """Eq. 1 then Eq. 2, with the velocity clamp and the box constraint. Plain loops."""
    N, D = x.shape
    xn = np.empty_like(x)
    vn = np.empty_like(v)
    for i in range(N):
        for d in range(D):
            vv = chi * (v[i, d] + c1 * u1[i, d] * (p[i, d] - x[i, d])
                        + c2 * u2[i, d] * (g[d] - x[i, d]))
            vv = min(max(vv, -vclamp[d]), vclamp[d])
            xx = x[i, d] + vv
            xx = min(max(xx, lo[d]), hi[d])
            vn[i, d] = vv
            xn[i, d] = xx
    return xn, vn


def elitist_mutation(x, f, g, nm, p_em, vr, ru, rn, lo, hi):
    """Elitist mutation of the nm particles with the largest misfit f.

    ru, rn: [nm][D] uniform and standard-normal draws, row k used for the k-th
    worst particle. Returns the new positions (velocities are not touched).
    """
    N, D = x.shape
    order = sorted(range(N), key=lambda i: (-f[i], i))
    xn = x.copy()
    for k in range(nm):
        l = order[k]
        for d in range(D):
            if ru[k, d] < p_em:
                val = g[d] + 0.1 * vr[d] * rn[k, d]
            else:
                val = g[d]
            xn[l, d] = min(max(val, lo[d]), hi[d])
    return xn
