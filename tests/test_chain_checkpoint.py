"""Checkpoint files of the HMC chain driver (host only)."""
import json

import numpy as np
import pytest
import torch


def test_checkpoint_round_trip(tmp_path):
    from paper_1611_00298_amd.hmc import load_checkpoint, save_checkpoint
    g = np.random.Generator(np.random.PCG64(5))
    U = torch.from_numpy(g.standard_normal((4, 2, 2, 2, 2, 3, 3)) + 1j * g.standard_normal((4, 2, 2, 2, 2, 3, 3)))
    rng = np.random.Generator(np.random.PCG64(11))
    rng.random(7)
    recs = [{"dH": 0.1, "accepted": True}, {"dH": -0.2, "accepted": False}]
    save_checkpoint(tmp_path, U, rng, recs)
    expect = rng.random(5)
    V = torch.zeros_like(U)
    rng2 = np.random.Generator(np.random.PCG64(999))
    got = load_checkpoint(tmp_path, V, rng2)
    assert got == recs
    assert torch.equal(U, V)
    assert np.array_equal(rng2.random(5), expect)   # the generator continues where it was saved


def test_checkpoint_absent_and_mismatch(tmp_path):
    from paper_1611_00298_amd.hmc import load_checkpoint, save_checkpoint
    U = torch.zeros((4, 2, 2, 2, 2, 3, 3), dtype=torch.complex128)
    rng = np.random.Generator(np.random.PCG64(1))
    assert load_checkpoint(tmp_path / "none", U, rng) is None
    save_checkpoint(tmp_path, U, rng, [])
    with pytest.raises(ValueError):
        load_checkpoint(tmp_path, torch.zeros((4, 2, 2, 2, 4, 3, 3), dtype=torch.complex128), rng)
    with pytest.raises(ValueError):
        load_checkpoint(tmp_path, U, np.random.Generator(np.random.MT19937(1)))
    doc = json.loads((tmp_path / "state.json").read_text())
    doc["n_done"] = 3
    (tmp_path / "state.json").write_text(json.dumps(doc))
    with pytest.raises(ValueError):
        load_checkpoint(tmp_path, U, rng)


def test_checkpoint_keeps_the_heatbath_interval(tmp_path):
    from paper_1611_00298_amd.hmc import load_checkpoint, save_checkpoint
    U = torch.zeros((4, 2, 2, 2, 2, 3, 3), dtype=torch.complex128)
    rng = np.random.Generator(np.random.PCG64(3))
    iv = {"lo": 0.9, "hi": 3.1, "n_poles": 7, "since": 2}
    save_checkpoint(tmp_path, U, rng, [{"dH": 0.0}], interval=iv)
    recs, got = load_checkpoint(tmp_path, U, rng, with_interval=True)
    assert recs == [{"dH": 0.0}] and got == iv
    save_checkpoint(tmp_path, U, rng, [])
    assert load_checkpoint(tmp_path, U, rng, with_interval=True) == ([], None)
