"""Checkpoint files of the load-path driver and of the network's training
state (host only: the files and their round trip; the GPU resume tests are
in test_gpu_solver.py and test_gpu_net.py)."""

import os

import numpy as np
import torch

import paper_2505_15535_amd as mfe
from paper_2505_15535_amd import learned


def test_load_path_checkpoint_round_trip(tmp_path):
    rng = np.random.default_rng(0)
    u = torch.from_numpy(rng.standard_normal(30))
    prev = torch.from_numpy(rng.standard_normal(30))
    path = tmp_path / "path.npz"
    mfe.save_checkpoint(path, u=u, prev=prev, t=0.5, h=0.25, h_cap=0.25, prev_h=None, n_steps=4)
    ck = mfe.load_checkpoint(path)
    assert np.array_equal(ck["u"], u.numpy()) and np.array_equal(ck["prev"], prev.numpy())
    assert float(ck["t"]) == 0.5 and float(ck["h"]) == 0.25 and int(ck["n_steps"]) == 4
    assert np.isnan(ck["prev_h"])
    # rewriting replaces the file whole; no temporary file is left behind
    mfe.save_checkpoint(path, u=u, prev=prev, t=0.75, h=0.25, h_cap=0.25, prev_h=0.25, n_steps=4)
    assert float(mfe.load_checkpoint(path)["t"]) == 0.75
    assert sorted(os.listdir(tmp_path)) == ["path.npz"]


def test_network_training_state_round_trip(tmp_path):
    net = learned.Net(learned.init_params(3), torch.device("cpu"), "linear")
    net.m.normal_()
    net.v.uniform_()
    net.step = 7
    path = tmp_path / "net.npz"
    net.save(path)
    back = learned.Net.load(path, torch.device("cpu"))
    assert back.variant == "linear" and back.step == 7
    assert torch.equal(back.w, net.w) and torch.equal(back.m, net.m) and torch.equal(back.v, net.v)


def test_shuffling_generator_state_survives_the_file(tmp_path):
    """The training checkpoint keeps the generator's state as JSON: the draws
    after a reload are the draws the uninterrupted generator makes."""
    import json
    rng = np.random.default_rng(11)
    rng.permutation(50)
    net = learned.Net(learned.init_params(0), torch.device("cpu"), "relu")
    path = tmp_path / "train.npz"
    net.save(path, epoch=3, rng=json.dumps(rng.bit_generator.state), hist=np.array([1.0, 0.5, 0.25]))
    ahead = rng.permutation(50)
    with np.load(path, allow_pickle=False) as f:
        back = np.random.default_rng(0)
        back.bit_generator.state = json.loads(str(f["rng"]))
        assert int(f["epoch"]) == 3 and list(f["hist"]) == [1.0, 0.5, 0.25]
    assert np.array_equal(back.permutation(50), ahead)
    assert sorted(os.listdir(tmp_path)) == ["train.npz"]
