"""Comparison helpers for GPU-vs-oracle parity tests."""
import numpy as np

# FP64 tolerance of one step from an identical state: the two sides use the same
# arithmetic order except the cell sums (tree vs sequential) and the libm of the
# transcendental functions, which differ by a few ulps.
RTOL = 1e-12


def assert_close(a, b, rtol=RTOL, what="", scale=None):
    """|a-b| <= rtol * max(|b|, scale); scale defaults to 1e-3 of max|b| (values that
    are sums of terms of that size cannot be compared more tightly)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if a.size == 0:
        return
    if scale is None:
        scale = max(np.abs(b).max(), 1e-300) * 1e-3
    err = np.abs(a - b)
    bad = err > rtol * np.maximum(np.abs(b), scale)
    assert not bad.any(), (what, int(bad.sum()), float((err / np.maximum(np.abs(b), scale)).max()),
                           np.argwhere(bad)[:5].ravel().tolist())


def cell_scale(psi_t):
    """Per-cell scale of each conserved component of the total state psi_t (rows of
    (rho, rho U, rho V, rho W, rho E)): rho, then the momentum scale
    rho * sqrt(2 E / rho) = sqrt(2 rho (rho E)) for the three momenta (a momentum
    component can vanish while the cell's momentum scale does not), then rho E."""
    t = np.abs(np.asarray(psi_t, np.float64))
    mom = np.sqrt(2.0 * t[:, 0] * t[:, 4])
    return np.stack([t[:, 0], mom, mom, mom, t[:, 4]], axis=1) + 1e-300


def compare_states(g, o, rtol=RTOL, label="", psi_t=None):
    """Integer parts bit-exact (counts, offsets = the sort permutation's cell
    structure), floating parts within rtol.  The wave part Psi_w is a difference of
    sums (absorbed minus resampled moments), so when psi_t is given it is compared
    against the scale of the same cell's total state (cell_scale), cell by cell."""
    assert g["step"] == o["step"], (label, g["step"], o["step"])
    assert np.array_equal(g["off"], o["off"]), (label, "offsets differ",
                                                np.flatnonzero(g["off"] != o["off"])[:10])
    assert_close(g["x"], o["x"], rtol, f"{label}:x")
    # A collision sets a velocity to m +- c_r n/2 (Appendix A) with unit vector n:
    # its rounding is relative to the particle's speed, so each component is
    # compared against |xi| of that particle (a component near zero carries the
    # rounding of the whole vector).
    speed = np.sqrt(np.asarray(o["u"], np.float64) ** 2 + np.asarray(o["v"], np.float64) ** 2
                    + np.asarray(o["w"], np.float64) ** 2)
    if speed.size:
        speed = np.maximum(speed, 1e-3 * speed.max() + 1e-300)
    for k in ("u", "v", "w"):
        assert_close(g[k], o[k], rtol, f"{label}:{k}", scale=speed)
    sc = None
    if psi_t is not None:
        sc = cell_scale(psi_t)
    assert_close(g["psi_w"], o["psi_w"], rtol, f"{label}:psi_w", scale=sc)
    assert_close(g["cr_max"], o["cr_max"], rtol, f"{label}:cr_max")


def compare_diag(g, o, label=""):
    for k in ("n_abs", "n_new", "n_cand", "n_coll"):
        assert np.array_equal(g[k], o[k]), (label, k, np.flatnonzero(g[k] != o[k])[:10])
    assert np.array_equal(g["n_inj"], o["n_inj"]), (label, g["n_inj"], o["n_inj"])
    assert g["n_out"] == o["n_out"], (label, g["n_out"], o["n_out"])
