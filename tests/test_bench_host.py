"""Host-side checks of the benchmark (no GPU): the one-GPU guard and the work
counts behind `value` and `roofline.achieved`, the latter against flops
counted by walking the loops of Alg. 1 and of the packed contraction on a
small workload."""
import itertools
import os
import subprocess
import sys

import bench
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def _walk_counts(nk, nao, naux, neo, nspin):
    """Flops by enumeration: every (q, k, L) block of Alg. 1 multiplies C^dagger (neo x nao) by the
    nao x nao block and the result by C (nao x neo); the contraction adds one product per kept
    (IJ, KL) and row."""
    wt = 0
    for _q, _k, _l in itertools.product(range(nk), range(nk), range(naux)):
        wt += 8 * (neo * nao * nao + neo * nao * neo)
    wt *= nspin
    npair = neo * (neo + 1) // 2
    rows = nk * naux
    tri = sum(1 for ij in range(npair) for kl in range(ij + 1))
    wc = nspin * rows * 2 * tri
    if nspin == 2:
        wc += rows * 2 * npair * npair
    return wt, wc


def test_work_counts_match_enumeration():
    for nspin in (1, 2):
        wl = synth.Workload("w", (2, 1, 1), 5, 3, 5, 5, nspin, 1.5, 1)
        wt, wc = bench.work_counts(wl)
        ref_t, ref_c = _walk_counts(wl.nk, wl.nao, wl.naux, wl.neo, nspin)
        assert wt == ref_t and wc == ref_c


def test_kernel_flops_sum_to_the_work():
    # the per-launch counts of stage 2 (i >= j half) and of the contractions add up to W_C and to
    # the stage-2 share of W_T as the library launches them (one stage-2 launch per q and spin)
    wl = synth.Workload("w", (2, 2, 1), 6, 4, 6, 6, 2, 1.5, 1)
    npair = wl.neo * (wl.neo + 1) // 2
    s8, s4 = bench.kernel_flops(wl, "contract_s8_x"), bench.kernel_flops(wl, "contract_s4_x")
    _, wc = bench.work_counts(wl)
    assert 2 * s8 + s4 == wc
    x2 = bench.kernel_flops(wl, "xform2_x")
    assert x2 == 8.0 * wl.nk * wl.naux * wl.nao * npair
    # one stage-1 launch per q covers both spins: N_k launches make the stage-1 share of W_T
    wt, _ = bench.work_counts(wl)
    x1 = bench.kernel_flops(wl, "xform1_x")
    assert wl.nk * x1 == 8.0 * wl.nk ** 2 * wl.naux * wl.nao ** 2 * wl.neo * wl.nspin
    # stage 2 over the full ij square (twice the i >= j count less the diagonal share), every q and spin
    full2 = 2 * x2 * wl.neo / (wl.neo + 1)
    assert abs(wl.nk * x1 + wl.nspin * wl.nk * full2 - wt) <= 1e-12 * wt


def test_coulomb_exchange_energies_match_einsum():
    """The benchmark's E_J / E_K from packed s8 / s4 blocks equal the plain
    einsum definitions on the unpacked oracle tensors (UHF, 3x2x1 mesh)."""
    import numpy as np
    import torch

    import bench
    import synth
    from oracle import kspace as ok
    wl = synth.Workload("ej", (3, 2, 1), 5, 12, 5, 5, 2, 1.5, 17)
    lat = synth.make_lattice(wl)
    lm = synth.three_index(wl)
    bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
    ck = bath["c_k"]
    g, _ = ok.transform_1e(ck, lat.dm_k)
    full = {"aa": ok.alg1_eri(lm, ck[0], wl.kmesh)[0], "bb": ok.alg1_eri(lm, ck[1], wl.kmesh)[0],
            "ab": ok.alg1_eri(lm, ck[0], wl.kmesh, ck[1])[0]}
    packed = {"aa": torch.from_numpy(ok.pack_s8(full["aa"])), "bb": torch.from_numpy(ok.pack_s8(full["bb"])),
              "ab": torch.from_numpy(ok.pack_s4(full["ab"]))}
    got = bench.coulomb_exchange_energies(packed, torch.from_numpy(g), chunk=37)
    for key, (sa, sb) in {"aa": (0, 0), "bb": (1, 1), "ab": (0, 1)}.items():
        ej = 0.5 * np.einsum("ijkl,ji,lk->", full[key], g[sa], g[sb])
        assert abs(got[key]["E_J"] - ej) < 1e-12 * max(1.0, abs(ej))
        if key != "ab":
            ek = 0.5 * np.einsum("ijkl,jk,li->", full[key], g[sa], g[sa])
            assert abs(got[key]["E_K"] - ek) < 1e-12 * max(1.0, abs(ek))
