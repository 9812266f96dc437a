"""Parity of the HIP float64 path with the oracle for the quark-line +
lepton-pair processes (a massless quark line with gluons and a photon/Z
decaying to a lepton pair; g ubar -> tau+ tau- g g ubar is the paper's DY+3j
subprocess, Sec. 3), run on an MI355X through the C ABI binding.

Tolerance and adjudication as in test_gpu_parity: relative 1e-12 per event,
events beyond it re-evaluated with the __float128 oracle (the GPU value within
1e-12 of it, or within 10x the spread of the quad result under 2^-52 input
perturbations).
"""
import numpy as np
import pytest

import oracle
from inputs import gluon_cuts, process_points
from test_gpu_parity import check_parity, get_me, gpu_me2, me_mod, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu

FAMILY = [("gux_taptamux", 8192, 1), ("gux_taptamgux", 4096, 2), ("gux_taptamggux", 4096, 3)]


@pytest.mark.parametrize("proc,n,seed", FAMILY)
def test_parity(me_mod, torch_cuda, proc, n, seed):
    print(f"[qew] {proc} n={n} seed={seed}", flush=True)
    mom = process_points(proc, n, seed)
    got = gpu_me2(me_mod, torch_cuda, proc, mom)
    rel = check_parity(proc, mom, got)
    print(f"[qew] {proc}: max rel {rel.max():.2e}, median {np.median(rel):.2e}", flush=True)


def test_parity_after_cuts(me_mod, torch_cuda):
    """The benchmark's points: jets (both gluons and the ubar) with p_T > 20 GeV,
    |eta| < 5 and Delta R > 0.4."""
    mom = process_points("gux_taptamggux", 8192, 4)
    mom = mom[gluon_cuts(mom)]
    print(f"[qew] gux_taptamggux after cuts: n={len(mom)}", flush=True)
    got = gpu_me2(me_mod, torch_cuda, "gux_taptamggux", mom)
    rel = check_parity("gux_taptamggux", mom, got)
    print(f"[qew] after cuts: max rel {rel.max():.2e}, median {np.median(rel):.2e}", flush=True)


@pytest.mark.parametrize("proc,n", [("gux_taptamux", 1), ("gux_taptamgux", 65), ("gux_taptamggux", 127),
                                    ("gux_taptamggux", 1)])
def test_ragged_sizes(me_mod, torch_cuda, proc, n):
    mom = process_points(proc, n, 123)
    check_parity(proc, mom, gpu_me2(me_mod, torch_cuda, proc, mom))


@pytest.mark.parametrize("proc", [p for p, _, _ in FAMILY])
def test_per_helicity(me_mod, torch_cuda, proc):
    torch = torch_cuda
    mom = process_points(proc, 64, 31)
    m = get_me(me_mod, proc)
    me2, qh = m.eval_helicities(torch.from_numpy(mom).cuda())
    torch.cuda.synchronize()
    want_me2, want_qh = oracle.me2(proc, mom, per_helicity=True)
    scale = want_qh.max(axis=1, keepdims=True)
    np.testing.assert_allclose(qh.cpu().numpy() / scale, want_qh / scale, rtol=0, atol=1e-12)
    np.testing.assert_allclose(me2.cpu().numpy(), want_me2, rtol=1e-12)


@pytest.mark.parametrize("proc,expect", [("gux_taptamux", 8), ("gux_taptamgux", 16), ("gux_taptamggux", 32)])
def test_helicity_filter(me_mod, torch_cuda, proc, expect):
    """Chirality conservation on both massless lines: a quarter of the
    helicities survive, and dropping the others changes nothing."""
    torch = torch_cuda
    m = get_me(me_mod, proc)
    assert len(m.good_helicities()) == expect
    t = torch.from_numpy(process_points(proc, 512, 77)).cuda()
    filtered = m.eval(t)
    full, qh = m.eval_helicities(t)
    torch.cuda.synchronize()
    torch.testing.assert_close(filtered, full, rtol=1e-14, atol=0)


@pytest.mark.parametrize("lanes", [2, 8, 32])
def test_helicity_lanes(me_mod, torch_cuda, lanes):
    torch = torch_cuda
    mom = process_points("gux_taptamggux", 1000, 41)
    t = torch.from_numpy(mom).cuda()
    m = me_mod.MatrixElement("gux_taptamggux")
    m.set_helicity_lanes(1)
    one = m.eval(t)
    m.set_helicity_lanes(lanes)
    many = m.eval(t)
    torch.cuda.synchronize()
    np.testing.assert_allclose(many.cpu().numpy(), one.cpu().numpy(), rtol=1e-13, atol=0)
    m.close()


def test_info(me_mod, torch_cuda):
    info = get_me(me_mod, "gux_taptamggux").info()
    assert info["npart"] == 7 and info["ncol"] == 6 and info["ndiag"] == 50
