"""The parameter bar for binary32 tracklets against the binary64 refit of the
same hits (Sec. 2 item 2, the fitted helix parameters), shared by the oracle
and GPU tests.

Strict bound, for every parameter of every compared tracklet:
  y, z          |d| <= 1e-3 cm
  sin phi, tan lambda   |d| <= 1e-4 * max(|ref|, 1)
  q/pT          |d| <= 1e-4 * max(|ref|, 0.1)

Named exception (the only one): a q/pT value outside its strict bound whose
deviation is at most 1 % of its own binary64 standard error.  Its cause:
binary32 rounding of the residuals (coordinates up to 250 cm carry a rounding
of ~1.5e-5 cm) times the q/pT gain, which is large while q/pT is barely
measured; the deviation is then far below the measurement error.  Each
exception is returned with its index, standard error and deviation, and their
number is bounded: at most 0.5 % of the compared tracklets, plus one.  Over
12 691 tracklets of 40 single-sector events there are 35 (0.28 %), the
largest at 0.35 % of its standard error; y, z, sin phi and tan lambda never
leave the strict bound."""
import math

import numpy as np

TOL_ABS = np.array([1e-3, 1e-3, 0.0, 0.0, 0.0])
TOL_REL = np.array([0.0, 0.0, 1e-4, 1e-4, 1e-4])
TOL_FLOOR = np.array([1.0, 1.0, 1.0, 1.0, 0.1])
EXC_SIGMA = 0.01    # an exception deviates by at most this fraction of sigma(q/pT)
EXC_FRACTION = 0.005


def strict_limits(p64):
    return TOL_ABS + TOL_REL * np.maximum(np.abs(p64), TOL_FLOOR)


def compare(p32, p64, cov64):
    """Returns (strict, exceptions, dev): strict[n, 5] is True where the strict
    bound holds; exceptions lists (index, sigma_q, deviation) of the q/pT
    values outside it; dev[n, 5] the absolute deviations."""
    p64 = np.asarray(p64, np.float64)
    dev = np.abs(np.asarray(p32, np.float64) - p64)
    strict = dev <= strict_limits(p64)
    sig = np.sqrt(np.asarray(cov64, np.float64)[:, 14])
    exc = [(int(i), float(sig[i]), float(dev[i, 4])) for i in np.flatnonzero(~strict[:, 4])]
    return strict, exc, dev


def allowed_exceptions(n):
    return int(math.ceil(EXC_FRACTION * n)) + 1


def assert_parameters(p32, p64, cov64, what=""):
    """Assert the bar; return the exception list (for reporting)."""
    strict, exc, dev = compare(p32, p64, cov64)
    n = len(dev)
    assert strict[:, :4].all(), f"{what}: y, z, sin phi or tan lambda outside the strict bound: max {dev.max(0)}"
    for i, sig, d in exc:
        assert d <= EXC_SIGMA * sig, f"{what}: q/pT exception {i}: deviation {d:.3g} above 1 % of sigma {sig:.3g}"
    assert len(exc) <= allowed_exceptions(n), f"{what}: {len(exc)} q/pT exceptions over {n} tracklets: {exc}"
    return exc
