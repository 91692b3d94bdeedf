"""Field comparison used by the GPU parity tests.

The parity metric is the relative L2 error over all polarisations and
samples, ||got - want|| / ||want||.  A norm alone would let a localised error
through (one wrong tile among 2^17 samples hardly moves it), so every
comparison also bounds each sample: |got_i - want_i| <= 20 * bar * rms(want),
i.e. no sample may be off by more than twenty times the rms error the bar
allows."""

import numpy as np

PEAK_FACTOR = 20.0


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def check(got, want, bar, what="", scale="rms"):
    """Assert rel(got, want) < bar and the per-sample bound; returns rel.

    scale: "rms" for noise-like fields (QAM, WDM, ASE), "max" for isolated
    pulses, whose error sits where the pulse is: there the bound is
    20 * bar * max|want| (a pulse of a few samples in a long window has an
    rms far below its peak)."""
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    err = rel(got, want)
    assert err < bar, f"{what} rel-L2 {err:.3e} >= {bar:.1e}"
    if scale == "max":
        ref = float(np.max(np.abs(want)))
    else:
        ref = float(np.linalg.norm(np.ravel(want)) / np.sqrt(want.size))
    diff = np.abs(np.ravel(got - want))
    peak = float(np.max(diff))
    assert peak <= PEAK_FACTOR * bar * ref, (
        f"{what} max per-sample error {peak:.3e} > {PEAK_FACTOR:g} x {bar:.1e} x {scale} "
        f"{ref:.3e} (at flat index {int(np.argmax(diff))})")
    return err
