"""Host-side persistence: the network's state file and the D-kernel autotune cache."""
import json

import numpy as np
import pytest
import torch

from paper_2202_07388_amd import nn_train, qdw


def test_network_state_round_trip(tmp_path):
    n = qdw.nn_weight_count()
    g = torch.Generator().manual_seed(3)
    w = torch.randn(2 * n, generator=g, dtype=torch.float32)
    adam = torch.randn(4 * n, generator=g, dtype=torch.float32)
    path = str(tmp_path / "net.safetensors")
    nn_train.save_state(path, w, adam, step=372, meta={"lattice": "16x8x8x8"})
    w2, adam2, step, md = nn_train.load_state(path)
    assert torch.equal(w2, w) and torch.equal(adam2, adam) and step == 372
    assert md["lattice"] == "16x8x8x8"
    nn_train.save_state(path, w)
    w3, adam3, step3, _ = nn_train.load_state(path)
    assert torch.equal(w3, w) and adam3 is None and step3 == 0


def test_network_state_rejects_foreign_files(tmp_path):
    from safetensors.torch import save_file
    path = str(tmp_path / "other.safetensors")
    save_file({"weights": torch.zeros(8)}, path, metadata={"format": "something-else"})
    with pytest.raises(ValueError):
        nn_train.load_state(path)
    save_file({"weights": torch.zeros(8)}, path, metadata={"format": nn_train.STATE_FORMAT})
    with pytest.raises(ValueError):
        nn_train.load_state(path)


def test_tune_cache_entries(tmp_path):
    path = str(tmp_path / "shapes.json")
    k64 = qdw.tune_key((64, 32, 32, 32), "f64", 1, "gpu A", "abc")
    k16 = qdw.tune_key((64, 32, 32, 32), "f16", 1, "gpu A", "abc")
    assert qdw.read_tune_cache(path, k64) is None          # no file yet
    qdw.write_tune_cache(path, k64, (64, 32, 0, 0, 1))
    qdw.write_tune_cache(path, k16, np.array([128, 2, 0, 0, 0]))
    assert qdw.read_tune_cache(path, k64) == (64, 32, 0, 0, 1)
    assert qdw.read_tune_cache(path, k16) == (128, 2, 0, 0, 0)
    qdw.write_tune_cache(path, k64, (128, 4, 1, 1, 0))     # replaced, the other kept
    assert qdw.read_tune_cache(path, k64) == (128, 4, 1, 1, 0)
    assert qdw.read_tune_cache(path, k16) == (128, 2, 0, 0, 0)
    # every part of the key separates entries
    for other in [qdw.tune_key((32, 32, 32, 32), "f64", 1, "gpu A", "abc"),
                  qdw.tune_key((64, 32, 32, 32), "f64", 4, "gpu A", "abc"),
                  qdw.tune_key((64, 32, 32, 32), "f64", 1, "gpu B", "abc"),
                  qdw.tune_key((64, 32, 32, 32), "f64", 1, "gpu A", "abd")]:
        assert qdw.read_tune_cache(path, other) is None
    # malformed files or entries read as misses
    with open(path, "w") as fh:
        json.dump({"version": 1, "entries": {k64: [1, 2, 3]}}, fh)
    assert qdw.read_tune_cache(path, k64) is None
    with open(path, "w") as fh:
        fh.write("{not json")
    assert qdw.read_tune_cache(path, k64) is None
    qdw.write_tune_cache(path, k64, (64, 32, 0, 0, 1))     # a broken file is replaced
    assert qdw.read_tune_cache(path, k64) == (64, 32, 0, 0, 1)


def test_kernel_version_tracks_the_sources():
    v = qdw.kernel_version()
    assert len(v) == 16 and v == qdw.kernel_version()
