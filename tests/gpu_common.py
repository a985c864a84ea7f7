"""Shared helpers of the GPU parity tests (inputs from ``synth``, expected
values from ``oracle``; nothing here computes any part of the method)."""
import functools

import numpy as np
import torch

import synth
from oracle import kspace as ok


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


@functools.lru_cache(maxsize=8)
def case(name, kmesh=None, nao=None, naux=None, nspin=None, seed=None):
    """Workload inputs plus the oracle's bath (by name, optionally reshaped)."""
    wl = synth.CONFIGS.get(name)
    if wl is None or kmesh is not None:
        base = wl or synth.CONFIGS["tiny"]
        wl = synth.Workload(name, tuple(kmesh or base.kmesh), nao or base.nao, naux or base.naux,
                            nao or base.nao, nao or base.nao, nspin or base.nspin, 1.5, seed or 4321)
    lat = synth.make_lattice(wl)
    lm = synth.three_index(wl)
    bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    return wl, lat, lm, bath
