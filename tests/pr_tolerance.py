"""Per-vertex tolerance of the PageRank parity tests (HIP path against the
oracle), derived from the iteration of Eq. (1).

Both sides iterate x <- (1-d)/n + d A x in FP64, where A[v][u] = 1/q(u) for
an arc u -> v (q = out-degree), and stop at the first iteration whose
largest change is at most thr.  They add the same positive terms in
different orders.

(i) Stopping distance.  With x* the fixed point and delta = x_k - x_(k-1)
the last change, x_k - x* = dA (x_(k-1) - x*), hence
x_k - x* = -(sum_{j>=1} (dA)^j) delta, and with |delta| <= thr everywhere
    |x_k(v) - x*(v)| <= thr * ((sum_{j>=1} (dA)^j) 1)(v) = thr * (p(v) - 1),
where p = 1 + dA p, i.e. p = n x* / (1 - d).  So p(v) is about 1/(1-d) for
an ordinary vertex and grows with a hub's rank.  Each side stops that close
to x*, so the two differ by at most 2 thr p(v) (p computed from the oracle's
ranks, at least 1).

(ii) Rounding.  Apart from the stop, the two differ only by the rounding of
their sums.  RT |pr(v)| with RT = 64 unit roundoffs allows a few tens of
ulps for it; at the thresholds tested the stopping term is at least as
large wherever a vertex has many in-arcs.

So |gpu(v) - oracle(v)| <= 2 thr max(1, n pr(v) / (1 - d)) + 64 u |pr(v)|,
with n the live vertices of the snapshot and u = 2^-53.
"""
import numpy as np

U = 2.0 ** -53
RT = 64 * U


def pr_tolerance(want, threshold, damping, n_live):
    want = np.abs(np.asarray(want, dtype=np.float64))
    if damping < 1.0:
        p = np.maximum(1.0, n_live * want / (1.0 - damping))
    else:
        p = np.ones_like(want)
    return 2.0 * threshold * p + RT * want


def assert_pr_close(got, want, threshold, damping, n_live, what=""):
    """Asserts the bound and returns the largest err / tolerance ratio."""
    got = np.asarray(got)
    want = np.asarray(want)
    tol = pr_tolerance(want, threshold, damping, n_live)
    err = np.abs(got - want)
    bad = err > tol
    assert not bad.any(), (what, np.nonzero(bad)[0][:8], got[bad][:8], want[bad][:8], (err / tol).max())
    return float((err / np.maximum(tol, 1e-300)).max())
