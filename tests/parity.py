"""Helpers that compare a device run with the oracle (test-only)."""
import numpy as np


def join_on_uid(a: dict, b: dict):
    """Indices (ia, ib) of records present exactly once on both sides, keyed by
    (instance, uid); duplicated uids (a 32-bit lineage collision) are left out."""
    def keyed(r):
        inst = r["inst"].astype(np.uint64)
        return r["uid"], inst

    ua, ia_inst = keyed(a)
    ub, ib_inst = keyed(b)
    ka = np.rec.fromarrays([ia_inst, ua])
    kb = np.rec.fromarrays([ib_inst, ub])
    va, ca = np.unique(ka, return_counts=True)
    vb, cb = np.unique(kb, return_counts=True)
    good = np.intersect1d(va[ca == 1], vb[cb == 1])
    sa = np.argsort(ka)
    sb = np.argsort(kb)
    pa = sa[np.searchsorted(ka[sa], good)]
    pb = sb[np.searchsorted(kb[sb], good)]
    return pa, pb, len(ka), len(kb)


def compare_records(dev: dict, ref: dict, fp64: bool, z_tol: float = 0.0):
    """Fraction of joined particles whose final state and event counts agree."""
    ia, ib, na, nb = join_on_uid(dev, ref)
    same = np.ones(len(ia), bool)
    if fp64 and z_tol > 0:
        same &= np.abs(dev["z"][ia] - ref["z"][ib]) <= z_tol
        same &= np.abs(dev["mu"][ia] - ref["mu"][ib]) <= z_tol
    else:
        same &= dev["z"][ia] == ref["z"][ib]
        same &= dev["mu"][ia] == ref["mu"][ib]
    same &= dev["E"][ia] == ref["E"][ib]
    same &= dev["layer"][ia] == ref["layer"][ib]
    same &= dev["spin"][ia] == ref["spin"][ib]
    same &= dev["gen"][ia] == ref["gen"][ib]
    same &= dev["dead"][ia] == (ref["dead"][ib] >= 0)
    if "ev" in dev:
        same &= np.all(dev["ev"][ia] == ref["ev"][ib], axis=1)
    if "w" in dev:
        same &= dev["w"][ia] == ref["w"][ib]
    return dict(joined=len(ia), n_dev=na, n_ref=nb, match=int(same.sum()),
                frac=float(same.mean()) if len(ia) else 1.0, bad=np.where(~same)[0][:10],
                ia=ia, ib=ib)


def rel_l1(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())
