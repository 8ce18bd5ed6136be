"""A kernel written against the public headers alone (include/kernelet.h,
include/kernelet_device.h; tests/user_kernel/), registered by its host
stub: over a 2-D grid with a ragged edge, every slicing plan gives the
bits of the unsliced run, and both equal a transpose (Section 4.1, index
rectification; Section 2.2, a slicing plan covers every workgroup once)."""
import ctypes
import os

import numpy as np
import pytest
import torch

import paper_1303_5164_amd as K

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "user_kernel", "libuser_kernel.so")


class Args(ctypes.Structure):
    _fields_ = [("inp", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("rows", ctypes.c_uint32), ("cols", ctypes.c_uint32)]


@pytest.fixture(scope="module")
def user():
    L = ctypes.CDLL(LIB)
    L.user_transpose_fn.restype = ctypes.c_void_p
    L.user_transpose_args_bytes.restype = ctypes.c_uint32
    assert L.user_transpose_args_bytes() == ctypes.sizeof(Args)
    rt = K.Runtime(0)
    d = K.builtin_desc("poly")           # a descriptor to fill in
    d.name = b"user_transpose"
    d.host_fn = L.user_transpose_fn()
    d.block_threads = 256
    d.args_bytes = ctypes.sizeof(Args)
    d.flags = 1
    k = rt.register(d)
    yield rt, k, L
    rt.close()


@pytest.mark.parametrize("rows,cols,slices", [(1000, 777, (0, 1, 7, 64, 1000)),
                                              (16, 4096, (0, 3, 255)),
                                              (33, 17, (0, 1, 2))])
def test_user_kernel_slices_to_unsliced_bits(user, rows, cols, slices):
    rt, k, _ = user
    dev = torch.device("cuda:0")
    g = torch.Generator().manual_seed(rows * 7 + cols)
    x = torch.rand(rows, cols, generator=g, dtype=torch.float32)
    inp = x.to(dev)
    grid = ((cols + 15) // 16, (rows + 15) // 16, 1)
    outs = []
    for s in slices:
        out = torch.full((cols, rows), -1.0, dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        print(f"# user kernel {rows}x{cols}, slice {s}", flush=True)
        j = rt.submit(k, grid, Args(inp.data_ptr(), out.data_ptr(), rows, cols))
        if s:
            n = rt.slice(j, s)
            assert n == -(-(grid[0] * grid[1]) // s)
        rt.schedule("fixed")
        rt.wait(j, 30_000_000_000)
        outs.append(out.cpu().numpy())
        rt.reap()
    ref = x.numpy().T
    assert np.array_equal(outs[0], ref)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
