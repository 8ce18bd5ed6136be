"""GPU tests of the surrogate path: the synthetic template kernels give the
same bits sliced, co-run and alone; a network trained on the device reaches
under 10% error on kernels it has not seen; the SURROGATE policy needs its
weights and runs a mix to the same bits as FIFO; with 64 synthetic types it
needs far fewer Markov solves than the Markov policy alone."""
import numpy as np
import pytest
import torch

import paper_1303_5164_amd as K
from paper_1303_5164_amd import _lib, profiles
from paper_1303_5164_amd import surrogate as S
from paper_1303_5164_amd import workloads as W
import synth

from gpu_util import result, small_mix

pytestmark = pytest.mark.gpu


def _synthk_args(dev, pattern, n_threads=1 << 16, iters=16, alu=8, log2_src=22):
    src = torch.from_numpy(synth.uniform_f32(0, synth.STREAM["synthk"], 1 << log2_src,
                                             0.5, 1.0)).to(dev)
    dst = torch.zeros(n_threads, dtype=torch.float32, device=dev)
    a = _lib.SynthkArgs(src.data_ptr(), dst.data_ptr(), (1 << log2_src) - 1, n_threads,
                        iters, alu, pattern, 0)
    return a, src, dst


@pytest.mark.parametrize("name", ["synthk_v32_l0", "synthk_v64_l16", "synthk_v256_l64"])
def test_synthk_sliced_and_corun_same_bits(name):
    dev = torch.device("cuda:0")
    prof = S.analytic_profile({"alu": 8, "pattern": 0, "vgpr": int(name.split("_")[1][1:]),
                               "lds_kb": int(name.split("_")[2][1:])})
    with K.Runtime(0) as rt:
        k1 = rt.register_builtin(name, prof)
        d2 = K.builtin_desc("synthk_v32_l0")
        d2.name = b"partner"
        k2 = rt.register(d2, S.analytic_profile({"alu": 2, "pattern": 2, "vgpr": 32,
                                                 "lds_kb": 0}))
        for pattern in (0, 1, 2):
            a, src, dst = _synthk_args(dev, pattern)
            grid = K.builtin_grid(name, a)
            assert grid == (256, 1, 1)
            outs = []
            for mode in ("alone", "sliced", "corun"):
                dst.zero_()
                pa, psrc, pdst = _synthk_args(dev, 2, alu=2)
                torch.cuda.synchronize()
                j = rt.submit(k1, grid, a)
                if mode != "alone":
                    rt.slice(j, 37)
                if mode == "corun":
                    j2 = rt.submit(k2, K.builtin_grid("synthk_v32_l0", pa), pa)
                    rt.slice(j2, 64)
                rt.schedule("fifo" if mode == "alone" else "fixed", blocking=True,
                            wait_done=True)
                rt.wait(j)
                outs.append(dst.clone())
                rt.reap()
            assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
            assert torch.isfinite(outs[0]).all().item()


def test_trained_surrogate_generalises_to_unseen_kernels():
    Xtr, Ttr, _ = S.dataset(0, 600, 12000, 0, 480)
    Xte, Tte, _ = S.dataset(0, 600, 3000, 480, 600)
    net = S.train(Xtr, Ttr, seed=0, epochs=30)
    y = net.forward(torch.from_numpy(Xte).cuda()).cpu().numpy()
    err = S.mape(y, Tte)
    print(f"held-out MAPE {err:.4f}", flush=True)
    assert err < 0.10


def test_surrogate_policy_same_bits_as_fifo():
    dev = torch.device("cuda:0")
    prof = profiles.load()
    insts = small_mix(dev)
    with K.Runtime(0, surrogate_topk=2) as rt:
        kids = {k: rt.register_builtin(k, prof[k]) for k in W.KERNELS}
        j = rt.submit(kids["poly"], insts[0].launches[0].grid, insts[0].launches[0].args)
        with pytest.raises(K.KerneletError) as e:
            rt.schedule("surrogate")
        assert e.value.code == -5                      # no weights loaded
        rt.schedule("fifo", blocking=True, wait_done=True)
        rt.reap()
        rt.set_surrogate(S.init_params(0))
        outs = {}
        for pol in ["fifo", "surrogate"]:
            for inst in insts:
                inst.reset()
            torch.cuda.synchronize()
            jobs = [W.submit(rt, kids, inst) for inst in insts]
            rt.schedule(pol, blocking=True, wait_done=True)
            for js in jobs:
                rt.wait(js[-1], 60_000_000_000)
            outs[pol] = [result(i) for i in insts]
            rt.reap()
        st = rt.stats()
    bad = [i.kind for i, a, b in zip(insts, outs["fifo"], outs["surrogate"])
           if not np.array_equal(a, b)]
    assert not bad, f"outputs differ from FIFO: {bad}"
    assert st["surrogate_pairs"] > 0 and st["surrogate_candidates"] > 0


def test_surrogate_gain_over_markov_on_64_synthetic_types():
    """What the trained network gains over the Markov model alone: the same
    256 jobs of 64 synthetic kernel types scheduled under MARKOV and under
    SURROGATE (network ranking every surviving pair, the Markov model
    judging the top 4).  The surrogate run needs far fewer Markov ratio
    searches, and every output equals FIFO's."""
    import argparse

    from paper_1303_5164_amd import synthmix
    res = synthmix.decide(argparse.Namespace(seed=7, types=64, jobs=256, topk=4))
    runs = {r["policy"]: r for r in res["runs"]}
    for pol in ("markov", "surrogate"):
        r = runs[pol]
        print(f"{pol}: decisions {r['decisions']} model solves {r['model_solves']} "
              f"decision ms {r['decision_ms_total']:.2f} wall ms {r['wall_ms']:.2f}", flush=True)
    assert res["mismatches_vs_fifo"] == 0
    m, s = runs["markov"], runs["surrogate"]
    assert m["decisions"] > 0 and s["decisions"] > 0
    assert s["pairs_scored"] > 0
    assert s["model_solves"] * 2 < m["model_solves"], (s["model_solves"], m["model_solves"])
