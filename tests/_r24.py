"""Shared comparison rule for float32 BP against the float64 oracle.

Bar: every posterior within 1e-4 relative, relative to max(|L64|, lambda_floor) with
lambda_floor = min_j |lambda_j|.  A shot is exempt only if the oracle's own trajectory, over the
iterations either side ran, passes within 1e-3 * lambda_floor of zero for some check-to-fault
message or posterior: float32 cannot be expected to reproduce the sign of such a value, and a
sign decides convergence, the iteration count and the hard decision.  Exempt shots are returned
so the tests can report them; any other disagreement fails.
"""
import numpy as np

REL = 1e-4
NEAR_ZERO = 1e-3


def floor_of(lam):
    return float(np.abs(lam).min())


def check_shot(oracle_mod, oc, lam, s, T, L32, gconv, giters, early_exit=True, hard32=None, alpha=0.625):
    """'ok' or 'exempt' (see the module docstring); raises AssertionError otherwise."""
    floor = floor_of(lam)
    conv, it, L64, h64 = oracle_mod.bp(oc, lam, s, T, alpha=alpha, early_exit=early_exit)
    same = bool(gconv) == conv and int(giters) == it
    if same:
        err = np.abs(np.asarray(L32, np.float64) - L64) / np.maximum(np.abs(L64), floor)
        ok = err.max() <= REL
        if ok and hard32 is not None:
            ok = bool((np.asarray(hard32) == h64).all())
        if ok:
            return "ok"
    mm = oracle_mod.bp_min_magnitude(oc, lam, s, max(int(giters), it), alpha=alpha)
    assert mm < NEAR_ZERO * floor, (
        f"float32 BP parts from the oracle on a shot whose trajectory stays {mm:.3e} away from zero "
        f"(exemption threshold {NEAR_ZERO * floor:.3e}); gpu conv={gconv} iters={giters}, oracle conv={conv} iters={it}")
    return "exempt"
