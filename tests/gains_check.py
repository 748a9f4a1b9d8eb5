"""Element-wise comparison of solved gains for the GPU parity tests."""
import numpy as np


def gain_err(a, b, n_corr=1):
    """Largest relative error over gain blocks: one block is the gain of one antenna in one
    direction (a complex value, or a 2x2 Jones matrix when n_corr = 4, compared in the
    Frobenius norm).  a and b hold the same blocks in the same order (either the library's
    [n_dir][n_ant][n_corr] layout or the oracle's, whose 2x2 matrices are contiguous)."""
    a = np.asarray(a, dtype=np.complex128).reshape(-1, n_corr)
    b = np.asarray(b, dtype=np.complex128).reshape(-1, n_corr)
    assert a.shape == b.shape, (a.shape, b.shape)
    num = np.linalg.norm(a - b, axis=1)
    den = np.linalg.norm(b, axis=1)
    return float(np.max(num / np.maximum(den, 1e-300)))


def stop_decision_is_clear(history, tol, n_stop, margin=0.1):
    """True when the oracle's stopping update n_stop (1-based) is decided with room to spare:
    the relative changes of the update before it and of the stopping update itself both lie
    more than `margin` (relative) away from tol.  FP32 gains carry a rounding of ~6e-8 of
    their norm, so a relative change of ~1e-6 is known to a few per cent; decisions closer
    to tol than that can legitimately differ between the FP32 kernels and the FP64 oracle."""
    idx = [n_stop - 1] + ([n_stop - 2] if n_stop >= 2 else [])
    return all(abs(history[i] / tol - 1.0) > margin for i in idx)


def oracle_stop(history, tol, max_iter):
    """Update count at which the oracle, run from the same start to a tighter tolerance,
    would have stopped at `tol` (its iterates are the same up to there)."""
    for i, h in enumerate(history):
        if h < tol:
            return i + 1
    return min(len(history), max_iter)
