"""Test helpers: hand an oracle setup to the library through gs_setup_explicit
(the same M^{-1} on both sides), and common tolerances.

Direction of data flow: oracle -> library only.  Nothing the library
computes is ever fed back into the oracle."""
import numpy as np


def oracle_levels(st):
    """gs_level_data list (as dicts) from an oracle.gemslr.Setup."""
    out = []
    for l, lv in enumerate(st.levels):
        d = {"d": lv.d, "block_ptr": np.asarray(lv.blocks, dtype=np.int64),
             "L": (lv.Lf.indptr, lv.Lf.indices, lv.Lf.data),
             "U": (lv.Uf.indptr, lv.Uf.indices, lv.Uf.data)}
        if lv.s > 0:
            d["E"] = (lv.E.indptr, lv.E.indices, lv.E.data)
            d["F"] = (lv.F.indptr, lv.F.indices, lv.F.data)
            d["W"] = lv.W
            d["H"] = lv.H
        out.append(d)
    return out


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
