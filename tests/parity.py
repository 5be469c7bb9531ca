"""Parity assertion shared by the GPU tests: the relative Frobenius error and
the max-abs / max-abs ratio of a GPU result against the oracle, both within
the bar (the relative Frobenius norm alone lets an error confined to the
small high-index coefficients pass)."""
import numpy as np


def errors(got, want):
    got = np.asarray(got)
    want = np.asarray(want)
    fro = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    mx = float(np.abs(got - want).max() / np.abs(want).max())
    return fro, mx


def check(got, want, bar=1e-12, label=""):
    fro, mx = errors(got, want)
    print(f"{label} rel err {fro:.3e} max-abs {mx:.3e}", flush=True)
    assert fro <= bar and mx <= bar, f"{label}: rel {fro:.3e}, max-abs {mx:.3e} (bar {bar:g})"
    return fro, mx
