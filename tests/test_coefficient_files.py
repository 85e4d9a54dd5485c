"""Coefficient files (save_coefficients / load_coefficients): the Lanczos
coefficients of (m, n) start vectors written to .npz and read back without
unpickling, for a resumed Sigma on another frequency grid.  Host only."""
import numpy as np
import pytest

import paper_2310_20103_amd as G


def _arrays(P=5, L=7, seed=3):
    rng = np.random.default_rng(seed)
    return dict(m=rng.integers(0, 40, P), n=rng.integers(0, 40, P),
                alpha=rng.standard_normal((P, L)), beta=rng.random((P, L)),
                norm2=rng.random(P), lens=rng.integers(1, L + 1, P))


def test_round_trip(tmp_path):
    a = _arrays()
    meta = {"poly_lo": 0.01, "poly_hi": 0.8, "poly_degree": 7, "grid": [24, 24, 24],
            "precision": "mixed"}
    path = tmp_path / "coeffs.npz"
    G.save_coefficients(path, a["m"], a["n"], a["alpha"], a["beta"], a["norm2"], a["lens"],
                        **meta)
    got, gmeta = G.load_coefficients(path)
    assert gmeta == meta
    for k, v in a.items():
        assert np.array_equal(got[k], v), k
    assert got["alpha"].dtype == np.float64 and got["lens"].dtype == np.int32
    with np.load(path, allow_pickle=False) as f:  # plain arrays only
        assert all(f[k].dtype != object for k in f.files)


def test_inconsistent_shapes_refused(tmp_path):
    a = _arrays()
    with pytest.raises(ValueError, match="inconsistent"):
        G.save_coefficients(tmp_path / "bad.npz", a["m"][:-1], a["n"], a["alpha"], a["beta"],
                            a["norm2"], a["lens"])
    with pytest.raises(ValueError, match="inconsistent"):
        G.save_coefficients(tmp_path / "bad.npz", a["m"], a["n"], a["alpha"], a["beta"][:, :-1],
                            a["norm2"], a["lens"])
