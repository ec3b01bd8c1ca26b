"""Checkpoint files on the CPU: a round trip is exact, the problem survives as
plain JSON, and malformed input is refused rather than guessed at."""

import numpy as np
import pytest

import problems
from paper_2110_10191_amd import checkpoint


def test_round_trip_is_exact(tmp_path):
    prm, P = problems.fm_torus(n1=24, n2=12, n3=4)
    path = str(tmp_path / "ck.npz")
    checkpoint.save(path, prm, P, 0.0123456789, t=1.5, step=7)
    ck = checkpoint.load(path)
    assert np.array_equal(ck.P, P) and ck.P.dtype == np.float64
    assert (ck.dt, ck.t, ck.step) == (0.0123456789, 1.5, 7)
    for k in ("n1", "n2", "n3", "a", "gam", "cfl", "x1min", "x1max", "bc", "recon", "precision", "floors"):
        assert ck.prm[k] == prm[k], k


def test_linear_modes_metadata_survives(tmp_path):
    prm, P = problems.linear_modes(n=8)
    path = str(tmp_path / "m.npz")
    checkpoint.save(path, prm, P, 0.01)
    ck = checkpoint.load(path)
    assert ck.prm["_modes"] == prm["_modes"]


def test_bad_input_is_refused(tmp_path):
    prm, P = problems.linear_modes(n=8)
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "a.npz"), prm, P[:, :-1], 0.01)
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "b.npz"), prm, P, 0.0)
    path = str(tmp_path / "c.npz")
    np.savez(path, format=np.int64(99), problem=np.array("{}"), P=P, dt=1.0, t=0.0, step=0)
    with pytest.raises(ValueError):
        checkpoint.load(path)
    # an archive holding a pickled object is not unpickled
    path = str(tmp_path / "d.npz")
    np.savez(path, format=np.int64(1), problem=np.array([{"n1": 8}], dtype=object), P=P, dt=1.0, t=0.0, step=0)
    with pytest.raises(ValueError):
        checkpoint.load(path)


def test_round_trip_with_electron_entropies(tmp_path):
    prm, P = problems.fm_torus(n1=24, n2=12, n3=4)
    E = problems.electron_scalars(P, prm["gam"], te_ti=0.5)
    path = str(tmp_path / "e.npz")
    checkpoint.save(path, prm, P, 0.01, E=E, heat=("kawazura", 0.0))
    ck = checkpoint.load(path)
    assert np.array_equal(ck.E, E) and ck.heat == ("kawazura", 0.0)
    plain = str(tmp_path / "p.npz")
    checkpoint.save(plain, prm, P, 0.01)
    assert checkpoint.load(plain).E is None and checkpoint.load(plain).heat is None
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "x.npz"), prm, P, 0.01, E=E[:, :-1], heat=("howes", 0.0))
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "y.npz"), prm, P, 0.01, E=E)
