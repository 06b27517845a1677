"""Edge-preserving regularisation (oracle, FP64).

Section 3.3: the smoothness term is a sum of a penalty phi over the first-order
pixel differences in both directions,

    Omega_1(x) = sum phi(x[n+1, m] - x[n, m]) + sum phi(x[n, m+1] - x[n, m]),

and the background term is Omega_0(x) = sum phi_{alpha_0}(x[n, m]).  The
difference ranges are not written out; this oracle uses non-periodic forward
differences (vertical rows n = 0..N-2, horizontal columns m = 0..N-2).  The
image is complex, so phi acts on the modulus of each difference.

Penalties phi(s), s = |t| >= 0, with the half-quadratic weight
w(s) = phi'(s)/s used by the gradient and by the majorise-minimise step:

* 'hyperbolic'  phi = sqrt(delta^2 + s^2)           w = 1/sqrt(delta^2 + s^2)
* 'huber'       phi = s^2 (s <= delta), 2 delta s - delta^2 otherwise
                (Section 3.3's Huber function with alpha = delta)
                                                     w = 2 (s <= delta), 2 delta/s
* 'quadratic'   phi = s^2 (Hunt's choice)            w = 2

Gradient convention: for a real-valued f of complex x, grad f = 2 df/d(conj x)
(real gradient packed as a complex array).  Then
grad sum phi(|D x|) = D^T (w(|Dx|) * Dx).
"""
from __future__ import annotations

import numpy as np

PHIS = ("hyperbolic", "huber", "quadratic")


def diff(x: np.ndarray):
    """(dv, dh): dv [..., N-1, N] vertical, dh [..., N, N-1] horizontal."""
    dv = x[..., 1:, :] - x[..., :-1, :]
    dh = x[..., :, 1:] - x[..., :, :-1]
    return dv, dh


def diff_adjoint(tv: np.ndarray, th: np.ndarray) -> np.ndarray:
    """D^T (tv, th): the adjoint of ``diff`` under <a, b> = sum conj(a) b."""
    N = th.shape[-2]
    out = np.zeros(th.shape[:-2] + (N, N), dtype=np.result_type(tv, th))
    out[..., 1:, :] += tv
    out[..., :-1, :] -= tv
    out[..., :, 1:] += th
    out[..., :, :-1] -= th
    return out


def phi(s: np.ndarray, delta: float, kind: str = "hyperbolic") -> np.ndarray:
    s = np.asarray(s, dtype=np.float64)
    if kind == "hyperbolic":
        return np.sqrt(delta * delta + s * s)
    if kind == "huber":
        return np.where(s <= delta, s * s, 2.0 * delta * s - delta * delta)
    if kind == "quadratic":
        return s * s
    raise ValueError(kind)


def weight(s: np.ndarray, delta: float, kind: str = "hyperbolic") -> np.ndarray:
    s = np.asarray(s, dtype=np.float64)
    if kind == "hyperbolic":
        return 1.0 / np.sqrt(delta * delta + s * s)
    if kind == "huber":
        with np.errstate(divide="ignore"):
            return np.where(s <= delta, 2.0, 2.0 * delta / np.maximum(s, delta))
    if kind == "quadratic":
        return np.full_like(s, 2.0)
    raise ValueError(kind)


def smooth_value(x: np.ndarray, delta: float, kind: str = "hyperbolic"):
    """Omega_1(x), summed over the last two axes."""
    dv, dh = diff(x)
    return (phi(np.abs(dv), delta, kind).sum(axis=(-2, -1))
            + phi(np.abs(dh), delta, kind).sum(axis=(-2, -1)))


def smooth_grad(x: np.ndarray, delta: float, kind: str = "hyperbolic"):
    """grad Omega_1 = D^T (w * D x)."""
    dv, dh = diff(x)
    return diff_adjoint(weight(np.abs(dv), delta, kind) * dv,
                        weight(np.abs(dh), delta, kind) * dh)


def smooth_curv(x: np.ndarray, d: np.ndarray, delta: float,
                kind: str = "hyperbolic"):
    """sum w(|Dx|) |Dd|^2, the curvature of the half-quadratic majorant."""
    dv, dh = diff(x)
    ev, eh = diff(d)
    return ((weight(np.abs(dv), delta, kind) * np.abs(ev) ** 2).sum(axis=(-2, -1))
            + (weight(np.abs(dh), delta, kind) * np.abs(eh) ** 2).sum(axis=(-2, -1)))


def background_value(x, alpha0, kind="huber"):
    """Omega_0(x) = sum phi_{alpha_0}(|x|)."""
    return phi(np.abs(x), alpha0, kind).sum(axis=(-2, -1))


def background_grad(x, alpha0, kind="huber"):
    return weight(np.abs(x), alpha0, kind) * x


def background_curv(x, d, alpha0, kind="huber"):
    return (weight(np.abs(x), alpha0, kind) * np.abs(d) ** 2).sum(axis=(-2, -1))
