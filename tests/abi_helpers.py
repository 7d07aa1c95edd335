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
    """Relative 2-norm difference ||a - b|| / ||b|| (reported beside the
    element-wise check, and used for solution vectors)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# Element-wise parity: every entry i must satisfy
#     |y_i - ref_i| <= tol * (|ref_i| + FLOOR * max_j |ref_j|),
# i.e. a relative error per entry, with a floor FLOOR * ||ref||_inf for
# entries that are tiny against the vector's scale (where rounding of the
# larger intermediate sums dominates).  A localised error -- one block, the
# last level, a few rows of a stage -- fails this even when the global norm
# hardly moves.
FLOOR = 1e-3


def elementwise_err(y, ref, floor=FLOOR):
    """max_i |y_i - ref_i| / (|ref_i| + floor * max_j |ref_j|)."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    scale = np.abs(ref) + floor * max(float(np.max(np.abs(ref))), 1e-300)
    return float(np.max(np.abs(y - ref) / scale))


def assert_close(y, ref, tol, floor=FLOOR, what=""):
    """Element-wise check of y against ref (see FLOOR); prints the
    element-wise, infinity-norm and 2-norm differences."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    assert y.shape == ref.shape, (y.shape, ref.shape)
    assert np.all(np.isfinite(y)), f"{what}: non-finite entries"
    e_el = elementwise_err(y, ref, floor)
    e_inf = float(np.max(np.abs(y - ref)) / max(float(np.max(np.abs(ref))), 1e-300))
    e_2 = relerr(y, ref)
    print(f"  {what} element-wise {e_el:.2e} (floor {floor:g}), inf-norm {e_inf:.2e}, "
          f"2-norm {e_2:.2e} (tol {tol:g})", flush=True)
    assert e_el <= tol, f"{what}: element-wise error {e_el:.3e} > {tol:g}"
    return e_el


# float32 / bfloat16 storage forms against the float64 oracle: entry by entry
# with a floor of 1e-2 ||ref||_inf (rounding of 2^-24 resp. 2^-9 per stored
# value, amplified through the dependent sweeps)
MIXED_FLOOR = 1e-2
MIXED_TOL = {"f32": 1e-2, "bf16": 1.0}
