"""Element-by-element comparison of GPU results with the FP64 oracle.

Two measures, both required below a tolerance by the parity tests:
  relmax       max |got - want| over the whole field / max |want|;
  site_relmax  for every 5d site (one s-slice of one 4d site: the last two axes
               are spin and colour), max |got - want| over its 12 complex
               components / max |want| over the same components.  The FP16
               storage keeps one norm per 5d site, so its error bound is
               relative to each site's own magnitude; a field whose site norms
               span many decades (a point-source Krylov vector) can only be
               checked this way.  A site where the oracle is exactly zero must
               be exactly zero on the GPU too.
"""
import numpy as np


def relmax(got, want):
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))


def site_relmax(got, want):
    d = np.abs(got - want).max(axis=(-2, -1))
    m = np.abs(want).max(axis=(-2, -1))
    zero = m == 0
    if np.any(d[zero] != 0):
        return float("inf")
    return float((d[~zero] / m[~zero]).max()) if np.any(~zero) else 0.0


def check(got, want, tol, what=""):
    """Assert both measures below tol; returns (relmax, site_relmax)."""
    g, s = relmax(got, want), site_relmax(got, want)
    assert g < tol and s < tol, (what, "global", g, "per site", s, "tol", tol)
    return g, s


def graded(psi, rng, decades=6):
    """psi with every 5d site scaled by 10^-u, u uniform in [0, decades)."""
    scale = 10.0 ** -rng.uniform(0, decades, size=psi.shape[:-2])
    return psi * scale[..., None, None]
