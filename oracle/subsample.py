"""Interface subsampling with interpolation along the interface lines.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).

Paper: Bihlo, Haynes & Walsh, arXiv:1504.00084, section 3.6: the interface
values can be estimated stochastically at every interface node, or at a
sample of them with the rest obtained by interpolation.  The paper points to
an optimal placement published elsewhere (not available here); this is the
equispaced reading:

- stride s (dividing both subdomain sizes): on a vertical interface line
  (i a multiple of (n_xi-1)/sub_xi, or the seam of a periodic xi axis) the
  nodes with j a multiple of s are estimated; on a horizontal line those with
  i a multiple of s; line crossings are always estimated;
- every other interface node takes the Keys cubic-convolution interpolant
  (a = -1/2) along its line through the known values at the multiples of s:
  the estimates, the boundary values at t^{n+1} where the line meets a
  Dirichlet side, Keys' end rule f(-s) = 3 f(0) - 3 f(s) + f(2s) beyond such
  a side, and the periodic image (plus the period for the coordinate that
  winds) across a periodic seam;
- its standard error is that of the same linear combination of independent
  estimates, sqrt(sum_k W_k^2 se_k^2) with W_k the total weight of estimate k
  (boundary values carry no error); its exit fraction is NaN.

Pinned by ``tests/test_oracle_subsample.py``.
"""
from __future__ import annotations

import math

import numpy as np

from . import Problem, interface_nodes


def keys_weights(t: float):
    """Keys' cubic-convolution weights (a = -1/2) of the points -1, 0, 1, 2."""
    return (((-0.5 * t + 1.0) * t - 0.5) * t, (1.5 * t - 2.5) * t * t + 1.0,
            ((-1.5 * t + 2.0) * t + 0.5) * t, (0.5 * t - 0.5) * t * t)


def check_stride(prob: Problem, stride: int):
    """Raise ValueError unless the stride divides both subdomain sizes and
    leaves at least two stride segments along every grid line (the fewest
    that Keys' end rule needs at a Dirichlet side)."""
    if stride < 1:
        raise ValueError("stride must be >= 1")
    if stride == 1:
        return
    Px = (prob.n_xi - 1) // prob.sub_xi
    Py = (prob.n_eta - 1) // prob.sub_eta
    if Px % stride or Py % stride:
        raise ValueError("stride %d does not divide the subdomain sizes %d x %d" % (stride, Px, Py))
    if (prob.n_xi - 1) // stride < 2 or (prob.n_eta - 1) // stride < 2:
        raise ValueError("stride %d leaves fewer than two segments along a grid line" % stride)


def sampled(prob: Problem, stride: int):
    """Boolean per interface rank: estimated by paths (True) or interpolated.
    Line crossings lie on multiples of the stride (it divides the subdomain
    sizes), so they are always estimated."""
    check_stride(prob, stride)
    I, J = interface_nodes(prob)
    if stride == 1:
        return np.ones(len(I), dtype=bool)
    Px = (prob.n_xi - 1) // prob.sub_xi
    Py = (prob.n_eta - 1) // prob.sub_eta
    on_v = (I % Px) == 0
    on_h = (J % Py) == 0
    return (on_v & (J % stride == 0)) | (on_h & (I % stride == 0))


def _side(prob: Problem, side: int, comp: int):
    n_xi, n_eta = prob.n_xi, prob.n_eta
    if side < 2:
        o = (side * 2 + comp) * n_eta
        return slice(o, o + n_eta)
    o = 4 * n_eta + ((side - 2) * 2 + comp) * n_xi
    return slice(o, o + n_xi)


def interpolate(prob: Problem, mean_x, mean_y, se_x, se_y, exit_frac, bnd_t1, stride: int):
    """Fill the non-sampled interface nodes of full-length result arrays
    (entries of sampled ranks are read, the others are overwritten)."""
    mean_x = np.array(mean_x, dtype=np.float64)
    mean_y = np.array(mean_y, dtype=np.float64)
    se_x = np.array(se_x, dtype=np.float64)
    se_y = np.array(se_y, dtype=np.float64)
    exit_frac = np.array(exit_frac, dtype=np.float64)
    check_stride(prob, stride)
    if stride == 1:
        return mean_x, mean_y, se_x, se_y, exit_frac
    bnd_t1 = np.asarray(bnd_t1, dtype=np.float64)
    I, J = interface_nodes(prob)
    rank = {(int(i), int(j)): r for r, (i, j) in enumerate(zip(I, J))}
    is_s = sampled(prob, stride)
    Px = (prob.n_xi - 1) // prob.sub_xi
    Py = (prob.n_eta - 1) // prob.sub_eta
    s = stride
    for r in range(len(I)):
        if is_s[r]:
            continue
        i, j = int(I[r]), int(J[r])
        vertical = i % Px == 0            # a non-sampled node lies on exactly one line
        n = prob.n_eta if vertical else prob.n_xi
        periodic = prob.periodic_eta if vertical else prob.periodic_xi
        period = (0.0, prob.Ly) if vertical else (prob.Lx, 0.0)   # offset of (x, y) over one period
        t = j if vertical else i

        def known(p):
            """(value x, value y, {rank: weight 1} or {}, offsets) at line position p."""
            off_x = off_y = 0.0
            if periodic:
                while p < 0:
                    p += n - 1
                    off_x -= period[0]
                    off_y -= period[1]
                while p > n - 2:
                    p -= n - 1
                    off_x += period[0]
                    off_y += period[1]
            elif p == 0 or p == n - 1:                 # a Dirichlet side at t^{n+1}
                side = (2 if p == 0 else 3) if vertical else (0 if p == 0 else 1)
                k = i if vertical else j
                return bnd_t1[_side(prob, side, 0)][k], bnd_t1[_side(prob, side, 1)][k], None
            q = rank[(i, p)] if vertical else rank[(p, j)]
            return mean_x[q] + off_x, mean_y[q] + off_y, q

        base = (t // s) * s
        w = keys_weights((t - base) / s)
        # stencil positions and weights, with Keys' end rule beyond a Dirichlet side
        terms = []
        for k in range(4):
            p = base + (k - 1) * s
            if not periodic and p < 0:
                terms += [(0, 3.0 * w[k]), (s, -3.0 * w[k]), (2 * s, w[k])]
            elif not periodic and p > n - 1:
                terms += [(n - 1, 3.0 * w[k]), (n - 1 - s, -3.0 * w[k]), (n - 1 - 2 * s, w[k])]
            else:
                terms.append((p, w[k]))
        vx = vy = 0.0
        W = {}
        for p, wk in terms:
            ax, ay, q = known(p)
            vx += wk * ax
            vy += wk * ay
            if q is not None:
                W[q] = W.get(q, 0.0) + wk
        mean_x[r] = vx
        mean_y[r] = vy
        se_x[r] = math.sqrt(sum(wq * wq * se_x[q] ** 2 for q, wq in W.items()))
        se_y[r] = math.sqrt(sum(wq * wq * se_y[q] ** 2 for q, wq in W.items()))
        exit_frac[r] = float("nan")
    return mean_x, mean_y, se_x, se_y, exit_frac
