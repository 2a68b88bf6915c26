"""Error metrics shared by the parity tests.

Reading of the tolerance (relative error on the log-value, <= 4e-15 in f64
and <= 2e-6 in f32): log I_v and log K_v pass through zero inside the
tested ranges, where a relative error is undefined for any algorithm.  The
gate therefore divides by max(|y|, 1 + sqrt(v^2 + x^2)), the size of the
log-value's sensitivity to relative perturbations of (v, x)
(|x dy/dx| + |v dy/dv| ~ sqrt(v^2 + x^2)).  Away from the zeros this is the
plain relative error.  The plain relative error is also computed and
reported.
"""
import numpy as np

TOL64 = 4e-15
TOL32 = 2e-6


def cond_err(y, hi, lo, v, x):
    """|y - ref| / max(|ref|, 1 + |(v, x)|) for finite references (others -> 0)."""
    y = np.asarray(y, dtype=np.float64)
    ref = hi + lo
    den = np.maximum(np.abs(hi), 1.0 + np.hypot(np.abs(v), x))
    with np.errstate(all="ignore"):
        e = np.abs((y - hi) - lo) / den
    return np.where(np.isfinite(hi), e, 0.0)


def rel_err(y, hi, lo):
    y = np.asarray(y, dtype=np.float64)
    with np.errstate(all="ignore"):
        e = np.abs((y - hi) - lo) / np.abs(hi)
    return np.where(np.isfinite(hi) & (hi != 0), e, 0.0)


def same_specials(y, hi):
    """Non-finite references must be matched exactly (NaN with NaN, +-inf)."""
    y = np.asarray(y, dtype=np.float64)
    bad = ~np.isfinite(hi)
    return np.array_equal(np.isnan(y[bad]), np.isnan(hi[bad])) and np.array_equal(
        y[bad][~np.isnan(hi[bad])], hi[bad][~np.isnan(hi[bad])]) and np.isfinite(y[~bad]).all()


def summary(e):
    e = np.asarray(e)
    return f"max={e.max():.3e} median={np.median(e):.3e} p99.99={np.quantile(e, 0.9999):.3e}"
