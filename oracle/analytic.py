"""Closed-form references for the Sod tube (test infrastructure only).

* Ballistic (collisionless, tau -> infinity) free streaming of two isotropic
  rest states (section "Numerical results", eq. ballistic): the continuum
  moments and the paper's density n_bal, plus the discrete-velocity version in
  which every polar node streams exactly.
* The ideal ultrarelativistic (P = e/3) Riemann problem, the tau -> 0 limit of
  the model: a left rarefaction and a right shock (standard relativistic
  hydrodynamics, used as the hydrodynamic-regime check of the same section),
  and the same problem seen from a frame in which both initial states move
  with a common velocity (moving initial states of eq. condinit).

Everything here is plain numpy/math written from the physics; nothing is
shared with the GPU path.
"""
import math

import numpy as np


# ---------------------------------------------------------------------------
# Ballistic regime
# ---------------------------------------------------------------------------

def ballistic_moments(z, t, left, right):
    """Continuum moments (N0, Nz, T00, T0z, Tzz) at z and t > 0.

    Two isotropic rest states (P, n, 0) stream freely from z < 0 and z > 0.
    A particle with polar cosine xi found at z came from z - xi t, i.e. from
    the left iff xi > s = z/t.  An isotropic rest state contributes n/2 dxi to
    N0 and e/2 dxi (e = 3P) to T00 per unit xi, so integrating over the
    side-dependent xi ranges gives the expressions below.
    """
    z = np.asarray(z, dtype=np.float64)
    s = np.clip(z / t, -1.0, 1.0)
    nL, nR = left[1], right[1]
    eL, eR = 3.0 * left[0], 3.0 * right[0]
    N0 = 0.5 * nL * (1 - s) + 0.5 * nR * (1 + s)
    Nz = 0.25 * (nL - nR) * (1 - s * s)
    T00 = 0.5 * eL * (1 - s) + 0.5 * eR * (1 + s)
    T0z = 0.25 * (eL - eR) * (1 - s * s)
    Tzz = eL * (1 - s ** 3) / 6.0 + eR * (1 + s ** 3) / 6.0
    return np.stack([N0, Nz, T00, T0z, Tzz])


def n_ballistic(z, t, nL=1.0, nR=0.125):
    """The paper's ballistic density profile (eq. ballistic)."""
    z = np.asarray(z, dtype=np.float64)
    s = np.clip(z / t, -1.0, 1.0)
    inner = np.sqrt(((nL + nR) / 2 - (nL - nR) / 2 * s) ** 2
                    - ((nL - nR) / 4) ** 2 * (1 - s * s) ** 2)
    s_raw = z / t
    return np.where(s_raw < -1, nL, np.where(s_raw > 1, nR, inner))


def ballistic_moments_discrete(z, t, left, right, xi, wxi):
    """Moments when each polar node xi_j streams exactly (no grid error).

    Same as ``ballistic_moments`` with the xi integral replaced by the
    Gauss-Legendre sum over the nodes: node j carries the left state at z iff
    z - xi_j t < 0.
    """
    z = np.asarray(z, dtype=np.float64)[None, :]
    xi = np.asarray(xi)[:, None]
    w = np.asarray(wxi)[:, None]
    from_left = (z - xi * t) < 0
    n = np.where(from_left, left[1], right[1])
    e = np.where(from_left, 3 * left[0], 3 * right[0])
    N0 = (0.5 * w * n).sum(0)
    Nz = (0.5 * w * n * xi).sum(0)
    T00 = (0.5 * w * e).sum(0)
    T0z = (0.5 * w * e * xi).sum(0)
    Tzz = (0.5 * w * e * xi * xi).sum(0)
    return np.stack([N0, Nz, T00, T0z, Tzz])


# ---------------------------------------------------------------------------
# Ideal P = e/3 Riemann problem (hydrodynamic limit)
# ---------------------------------------------------------------------------
CS = 1.0 / math.sqrt(3.0)  # sound speed of the ultrarelativistic gas


def _rarefaction_velocity(e, eL):
    # Along the left-moving fan the Riemann invariant atanh(v) + (sqrt(3)/4) ln e
    # is constant; the left state is at rest.
    return math.tanh(math.sqrt(3.0) / 4.0 * math.log(eL / e))


def _shock_velocity(e, eR):
    # Taub jump conditions for P = e/3 into a state at rest: relative velocity
    # of the post-shock fluid.
    P, PR = e / 3.0, eR / 3.0
    return math.sqrt((P - PR) * (e - eR) / ((eR + P) * (e + PR)))


def riemann_star(left, right):
    """Star state of the Sod problem: dict(e, v, V, nL, nR, tail)."""
    eL, eR = 3.0 * left[0], 3.0 * right[0]
    lo, hi = eR, eL
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _rarefaction_velocity(mid, eL) > _shock_velocity(mid, eR):
            lo = mid
        else:
            hi = mid
    e = 0.5 * (lo + hi)
    v = _rarefaction_velocity(e, eL)
    g = 1.0 / math.sqrt(1 - v * v)
    # shock speed from energy conservation across the front, right state at rest
    P = e / 3.0
    T00 = (e + P) * g * g - P
    T0z = (e + P) * g * g * v
    V = T0z / (T00 - eR)
    nR_star = right[1] * V / (g * (V - v))
    nL_star = left[1] * (e / eL) ** 0.75   # isentropic: n ~ e^(3/4)
    tail = (v - CS) / (1 - v * CS)
    return dict(e=e, v=v, V=V, nL=nL_star, nR=nR_star, tail=tail, P=P, T00=T00, T0z=T0z)


def riemann_profile(z, t, left, right):
    """(e, v, n) of the ideal Riemann solution at z, t > 0."""
    st = riemann_star(left, right)
    eL, eR = 3.0 * left[0], 3.0 * right[0]
    z = np.asarray(z, dtype=np.float64)
    s = z / t
    e = np.empty_like(s); v = np.empty_like(s); n = np.empty_like(s)
    for k, sk in enumerate(s):
        if sk < -CS:
            e[k], v[k], n[k] = eL, 0.0, left[1]
        elif sk < st["tail"]:
            vk = (sk + CS) / (1 + sk * CS)
            ek = eL * math.exp(-4.0 / math.sqrt(3.0) * math.atanh(vk))
            e[k], v[k], n[k] = ek, vk, left[1] * (ek / eL) ** 0.75
        elif sk < st["v"]:
            e[k], v[k], n[k] = st["e"], st["v"], st["nL"]
        elif sk < st["V"]:
            e[k], v[k], n[k] = st["e"], st["v"], st["nR"]
        else:
            e[k], v[k], n[k] = eR, 0.0, right[1]
    return e, v, n


# ---------------------------------------------------------------------------
# Boosted frame
# ---------------------------------------------------------------------------
def boost_velocity(v, w):
    """Velocity of a fluid moving at v in a frame that itself moves at w."""
    return (v + w) / (1.0 + v * w)


def riemann_profile_boosted(z, t, left, right, w):
    """(e, v, n) at z, t > 0 of the Riemann problem whose states, given in their
    common rest frame as (P, n, 0), both move with velocity w.

    The initial jump sits at z = 0, t = 0 in every frame, so the solution is a
    function of z/t only: the lab state at s = z/t is the rest-frame state at
    s' = (s - w)/(1 - s w), with the rest-frame scalars e and n unchanged and
    the fluid velocity boosted by w.
    """
    s = np.asarray(z, dtype=np.float64) / t
    sp = (s - w) / (1.0 - s * w)
    e, v, n = riemann_profile(sp, 1.0, left, right)
    return e, boost_velocity(v, w), n
