"""GPU runs of kernels written without slicing, made sliceable by rewriting
their device IR (Section 4.1) and registered from the code object through
the C ABI (kernelet_register_image): whole, in slices of several sizes with
ragged tails, and co-scheduled with a built-in kernel, every workgroup of
the original 2-D or 3-D grid runs once with its original indices and grid
size, and the paper's matrix-addition example gives A + B exactly."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1303_5164_amd as K
from paper_1303_5164_amd import build as B
from paper_1303_5164_amd import profiles
from paper_1303_5164_amd import workloads as W

from gpu_util import result

pytestmark = pytest.mark.gpu


class MatAddArgs(C.Structure):
    _fields_ = [("a", C.c_void_p), ("b", C.c_void_p), ("c", C.c_void_p), ("n", C.c_uint32)]


class Visit3dArgs(C.Structure):
    _fields_ = [("visits", C.c_void_p), ("dims", C.c_void_p), ("n", C.c_uint32)]


def _image():
    with open(B.PLAIN_IMAGE, "rb") as f:
        return f.read()


def _run(rt, k, grid, args, slice_wgs, policy="fixed"):
    torch.cuda.synchronize()
    j = rt.submit(k, grid, args)
    if slice_wgs:
        rt.slice(j, slice_wgs)
    rt.schedule(policy, blocking=True, wait_done=True)
    rt.wait(j, 60_000_000_000)
    torch.cuda.synchronize()
    rt.reap()


def test_matrix_add_sliced_is_exact():
    dev = torch.device("cuda:0")
    n = 1000                                   # 63 x 63 blocks, ragged edges
    a = synth.uniform_f32(3, synth.STREAM["poly_x"], n * n, -1.0, 1.0)
    b = synth.uniform_f32(4, synth.STREAM["poly_x"], n * n, -1.0, 1.0)
    want = (a + b).reshape(n, n)               # fp32 addition, element by element
    da, db = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    dc = torch.empty(n * n, dtype=torch.float32, device=dev)
    args = MatAddArgs(da.data_ptr(), db.data_ptr(), dc.data_ptr(), n)
    grid = (63, 63, 1)
    with K.Runtime(0) as rt:
        k = rt.register_image("plain_matadd", _image(), "kl_plain_matadd", C.sizeof(MatAddArgs))
        info = rt.kernel_info(k)
        assert info["max_wg_per_cu"] >= 1 and info["lds_bytes"] == 0
        for policy, s in [("fifo", 0), ("fixed", 1), ("fixed", 7), ("fixed", 1000),
                          ("fixed", 3969)]:
            print(f"matadd {policy} slice {s}", flush=True)
            dc.fill_(float("nan"))
            _run(rt, k, grid, args, s, policy)
            got = dc.cpu().numpy().reshape(n, n)
            assert np.array_equal(got, want), f"{policy} slice {s}"


@pytest.mark.parametrize("grid,slice_wgs", [((7, 5, 3), 4), ((1, 1, 1), 1),
                                            ((33, 2, 2), 64), ((256, 4, 1), 100)])
def test_every_block_once_with_the_original_grid(grid, slice_wgs):
    dev = torch.device("cuda:0")
    nwg = grid[0] * grid[1] * grid[2]
    visits = torch.zeros(nwg, dtype=torch.int32, device=dev)
    dims = torch.zeros(4, dtype=torch.int32, device=dev)
    args = Visit3dArgs(visits.data_ptr(), dims.data_ptr(), nwg)
    with K.Runtime(0) as rt:
        k = rt.register_image("plain_visit3d", _image(), "kl_plain_visit3d",
                              C.sizeof(Visit3dArgs))
        print(f"visit3d grid {grid} slice {slice_wgs}", flush=True)
        _run(rt, k, grid, args, slice_wgs)
    assert torch.equal(visits.cpu(), torch.ones(nwg, dtype=torch.int32))
    assert dims.cpu().tolist() == list(grid) + [0]


def test_coscheduled_with_a_builtin_kernel_under_the_markov_policy():
    """The rewritten kernel (with a first-order profile) and the built-in
    polynomial kernel, both sliced, scheduled by the Markov model."""
    dev = torch.device("cuda:0")
    grid = (64, 32, 2)
    nwg = grid[0] * grid[1] * grid[2]
    visits = torch.zeros(nwg, dtype=torch.int32, device=dev)
    dims = torch.zeros(4, dtype=torch.int32, device=dev)
    args = Visit3dArgs(visits.data_ptr(), dims.data_ptr(), nwg)
    h = synth.poly(0, n=1 << 18)
    inst = W.build("poly", W.device_inputs("poly", h, dev), {}, dev)
    prof = profiles.load()
    with K.Runtime(0, use_prune=0) as rt:
        kids = {kk: rt.register_builtin(kk, prof[kk]) for kk in W.KERNELS}
        k = rt.register_image("plain_visit3d", _image(), "kl_plain_visit3d",
                              C.sizeof(Visit3dArgs), dict(prof["gather"], instr_per_wave=30.0))
        torch.cuda.synchronize()
        j1 = rt.submit(k, grid, args)
        rt.slice(j1, 512)
        j2 = W.submit(rt, kids, inst)[0]
        rt.slice(j2, 256)
        rt.schedule("markov", blocking=True, wait_done=True)
        for j in (j1, j2):
            rt.wait(j, 60_000_000_000)
        torch.cuda.synchronize()
        dec = rt.decisions()
    assert torch.equal(visits.cpu(), torch.ones(nwg, dtype=torch.int32))
    assert dims.cpu().tolist() == list(grid) + [0]
    assert np.array_equal(result(inst), oracle.poly_f32_horner(h["x"], h["coef"]))
    assert dec, "no decision was logged"
