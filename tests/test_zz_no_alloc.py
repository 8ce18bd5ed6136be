"""The training step that allocates nothing (kernelet_mlp_train_step_noalloc,
its workspace a static device array of the library) against the step with a
caller workspace (kernelet_mlp_train_step), through the C ABI: parameters,
Adam moments and gradients bit for bit, over two calls in a row, the second
with a smaller batch than the first, so the first call's leftovers in the
shared array must not reach the second's results."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from paper_1303_5164_amd import _lib
from paper_1303_5164_amd import surrogate as S

pytestmark = pytest.mark.gpu


def _data(n, seed):
    x = synth.uniform_f32(seed, synth.STREAM["synthk"], n * 16, -1.0, 1.0).reshape(n, 16)
    t = (np.cos(2.0 * x[:, 0]) - x[:, 1] * x[:, 4] + 0.25 * x[:, 2]).astype(np.float32)
    order = np.argsort(synth.raw_u64(seed, synth.STREAM["mlp_shuffle"], n), kind="stable")
    return x, t, order.astype(np.int32)


class _State:
    def __init__(self, theta, dev):
        self.p = torch.from_numpy(theta.copy()).to(dev)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.g = torch.empty_like(self.p)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_max_batch_is_stated():
    assert _lib.lib().kernelet_mlp_noalloc_max_batch() == 4096


def test_batch_above_the_maximum_is_refused():
    L = _lib.lib()
    dev = torch.device("cuda:0")
    st = _State(S.init_params(0), dev)
    x = torch.zeros((8, 16), dtype=torch.float32, device=dev)
    t = torch.zeros(8, dtype=torch.float32, device=dev)
    big = L.kernelet_mlp_noalloc_max_batch() + 1
    rc = L.kernelet_mlp_train_step_noalloc(
        st.p.data_ptr(), None, None, x.data_ptr(), t.data_ptr(), None, big, 0,
        C.c_float(0.0), st.g.data_ptr(), _stream())
    assert rc == -1  # KL_EINVAL
    assert b"exceeds the maximum" in L.kernelet_last_error()


@pytest.mark.parametrize("seed", [0, 7])
def test_noalloc_step_equals_workspace_step_on_two_calls(seed):
    L = _lib.lib()
    dev = torch.device("cuda:0")
    maxb = int(L.kernelet_mlp_noalloc_max_batch())
    n = maxb + 500
    x, t, order = _data(n, seed)
    xd = torch.from_numpy(x).to(dev)
    td = torch.from_numpy(t).to(dev)
    theta = S.init_params(seed + 11)
    ref, got = _State(theta, dev), _State(theta, dev)
    # the larger call first (the full array), then a smaller ragged one
    for step, (lo, batch) in enumerate([(0, maxb), (100, 333)], start=1):
        idx = torch.from_numpy(np.ascontiguousarray(order[lo:lo + batch])).to(dev)
        ws = torch.empty(int(L.kernelet_mlp_workspace_floats(batch)), dtype=torch.float32,
                         device=dev)
        print(f"no-alloc step {step}: seed {seed}, batch {batch}", flush=True)
        _lib.check("kernelet_mlp_train_step", L.kernelet_mlp_train_step(
            ref.p.data_ptr(), ref.m.data_ptr(), ref.v.data_ptr(), xd.data_ptr(),
            td.data_ptr(), idx.data_ptr(), batch, step, C.c_float(1e-3), ref.g.data_ptr(),
            ws.data_ptr(), _stream()))
        _lib.check("kernelet_mlp_train_step_noalloc", L.kernelet_mlp_train_step_noalloc(
            got.p.data_ptr(), got.m.data_ptr(), got.v.data_ptr(), xd.data_ptr(),
            td.data_ptr(), idx.data_ptr(), batch, step, C.c_float(1e-3), got.g.data_ptr(),
            _stream()))
        torch.cuda.synchronize()
        for name in ("g", "p", "m", "v"):
            a = getattr(ref, name).cpu().numpy()
            b = getattr(got, name).cpu().numpy()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (step, name)
        assert np.isfinite(ref.g.cpu().numpy()).all() and ref.g.abs().sum().item() > 0
        del ws
