"""Shared test helpers: oracle runs on generator inputs, tolerance checks."""
import numpy as np

from oracle import crown, pipeline as opipe
from paper_2512_11087_amd import workloads as wl

REL = 1e-5   # parity band: |gpu - oracle| <= REL * max(|oracle|, 1)


def assert_close(gpu, ref, rel=REL, what=""):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    both_inf = np.isinf(gpu) & np.isinf(ref) & (np.sign(gpu) == np.sign(ref))
    err = np.where(both_inf, 0.0, np.abs(gpu - ref))
    tol = rel * np.maximum(np.abs(np.where(np.isinf(ref), 1.0, ref)), 1.0)
    bad = ~(err <= tol)
    if bad.any():
        i = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside {rel} rel; first at {tuple(i)}:"
                             f" gpu={gpu[tuple(i)]!r} oracle={ref[tuple(i)]!r}")
    return float(np.max(np.where(both_inf, 0.0, err / np.maximum(np.abs(np.where(np.isinf(ref), 1.0, ref)), 1.0)), initial=0.0))


class OracleProp:
    """Oracle-side state of one workload: dense layers and root pass."""

    def __init__(self, w, alpha0=0.5):
        self.w = w
        self.layers = crown.dense_layers(w.net)
        self.root = crown.root_pass(self.layers, w.lo0, w.hi0, alpha0)
        _, _, _, _, self.l0, self.u0 = self.root.stacked()

    def unstable(self):
        return np.nonzero((self.l0 < 0) & (self.u0 > 0))[0]

    def run(self, sp, lo=None, hi=None, cfg=opipe.Config()):
        B = sp.B
        if lo is None:
            lo = np.broadcast_to(self.w.lo0, (B, self.w.net.n_in)).astype(np.float64)
            hi = np.broadcast_to(self.w.hi0, (B, self.w.net.n_in)).astype(np.float64)
        return opipe.run(self.layers, self.root, self.w.C, self.w.t, lo, hi, sp.neuron, sp.sign,
                         sp.count, cfg)


def subset_splits(sp, idx):
    return wl.Splits(sp.neuron[idx], sp.sign[idx], sp.count[idx])
