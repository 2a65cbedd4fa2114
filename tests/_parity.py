"""Shared force-parity measures of the GPU tests (imported by the test modules; no tests here).

Two error measures, both asserted by check():
* rms relative, over the listed i: e_a = sqrt(mean_i |a_i - a_i^ref|^2 / |a_i^ref|^2), likewise
  for the jerk and the potential;
* per row, against the size of the row's terms: |a_i - a_i^ref| / sa_i with
  sa_i = sum_{j != i} m_j |d| s^-3/2, and |k_i - k_i^ref| / sk_i with
  sk_i = sum_{j != i} m_j (|u| s^-3/2 + 3 |d.u| |d| s^-5/2) (oracle.force_scale); the potential
  terms share one sign, so its per-row relative error is that measure already.  A sum of terms
  rounded to relative u is off by at most about u times that scale however much the pulls
  cancel, so no row, including one near the centre whose pulls cancel to a tiny |a|, may exceed
  the target on it.
The same tolerance bounds the rms and every row.
"""
import numpy as np

import oracle

TOL = {"fp32": (2e-6, 1e-5, 2e-6), "ds": (1e-11, 1e-10, 1e-11), "fp64": (1e-13, 1e-13, 1e-13),
       "fp32all": (1e-5, 1e-4, 1e-5)}


def rms_rel(got, ref):
    got = np.asarray(got); ref = np.asarray(ref)
    if got.ndim == 1:
        return float(np.sqrt(np.mean(((got - ref) / ref) ** 2)))
    num = np.sum((got - ref) ** 2, axis=1)
    den = np.sum(ref ** 2, axis=1)
    return float(np.sqrt(np.mean(num / den)))


def row_errors(got, ref, scale):
    """Per-row errors: |da_i| / sa_i, |dk_i| / sk_i, |dphi_i| / |phi_i|."""
    sa, sk = scale
    ra = np.linalg.norm(np.asarray(got[0]) - ref[0], axis=1) / sa
    rk = np.linalg.norm(np.asarray(got[1]) - ref[1], axis=1) / sk
    rp = np.abs(np.asarray(got[2]) - ref[2]) / np.abs(ref[2])
    return ra, rk, rp


def check(prec, got, ref, scale, label=""):
    """rms relative errors and every row's scaled error within the tolerances of `prec`."""
    ta, tk, tp = TOL[prec]
    ea, ek, ep = rms_rel(got[0], ref[0]), rms_rel(got[1], ref[1]), rms_rel(got[2], ref[2])
    ra, rk, rp = row_errors(got, ref, scale)
    print(f"{label} {prec}: rows {len(ra)}: e_acc={ea:.3e} e_jerk={ek:.3e} e_pot={ep:.3e}; "
          f"worst row acc {ra.max():.3e} (row {int(ra.argmax())}) jerk {rk.max():.3e} "
          f"pot {rp.max():.3e}", flush=True)
    assert ea <= ta and ek <= tk and ep <= tp, (ea, ek, ep)
    assert ra.max() <= ta and rk.max() <= tk and rp.max() <= tp, \
        (int(ra.argmax()), ra.max(), int(rk.argmax()), rk.max(), int(rp.argmax()), rp.max())


def reference(x, v, m, eps2, idx=None):
    """Oracle forces and per-row term scales of the listed i."""
    return oracle.force(x, v, m, eps2, idx=idx), oracle.force_scale(x, v, m, eps2, idx=idx)


def stratified_rows(n, block, seed):
    """One seeded row from every `block` consecutive rows, plus the first and the last row."""
    nb = (n + block - 1) // block
    r = np.random.default_rng(seed).integers(0, block, nb)
    rows = np.minimum(np.arange(nb) * block + r, n - 1)
    return np.unique(np.concatenate([[0], rows, [n - 1]])).astype(np.int64)
