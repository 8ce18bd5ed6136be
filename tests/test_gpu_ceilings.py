"""GPU runs of the ceiling probes (the FP32 FMA loop, the FP32
matrix-instruction loop and the HBM read stream the kernels' roofs are
measured with): whole and sliced with a ragged tail, every thread writes the
value its chains, accumulators or sums reach, exactly (integers below 2^24
in FP32)."""
import pytest
import torch

import paper_1303_5164_amd as K
from paper_1303_5164_amd import _lib
from paper_1303_5164_amd import calibrate as CAL

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,iters", [("ceil_fma", 1000), ("ceil_mfma", 500)])
@pytest.mark.parametrize("slice_wgs", [0, 8])
def test_ceiling_probes_write_exact_values(kind, iters, slice_wgs):
    dev = torch.device("cuda:0")
    n_wg = 37
    buf = torch.full((n_wg * 256,), -1.0, dtype=torch.float32, device=dev)
    args = _lib.CeilingArgs(buf.data_ptr(), 1.0, 1.0, n_wg, iters)
    with K.Runtime(0) as rt:
        k = rt.register_builtin(kind)
        torch.cuda.synchronize()
        print(f"{kind} iters {iters} slice {slice_wgs}", flush=True)
        j = rt.submit(k, (n_wg, 1, 1), args)
        if slice_wgs:
            rt.slice(j, slice_wgs)
        rt.schedule("fixed" if slice_wgs else "fifo", blocking=True, wait_done=True)
        rt.wait(j, 60_000_000_000)
        torch.cuda.synchronize()
    want = CAL.ceiling_expected(kind, iters)
    assert torch.all(buf.cpu() == want), (kind, buf.cpu()[:4].tolist(), want)


@pytest.mark.parametrize("slice_wgs", [0, 8])
def test_read_probe_sums_exactly(slice_wgs):
    """Each thread sums its 4 * per_thread floats; with src[i] = i mod 7 the
    sums are small integers the host computes the same way."""
    dev = torch.device("cuda:0")
    n_wg, per = 37, 16
    n = n_wg * 256 * per * 4
    src = (torch.arange(n, dtype=torch.int64, device=dev) % 7).to(torch.float32)
    out = torch.full((n_wg * 256,), -1.0, dtype=torch.float32, device=dev)
    args = _lib.ReadArgs(src.data_ptr(), out.data_ptr(), n_wg, per)
    with K.Runtime(0) as rt:
        k = rt.register_builtin("ceil_read")
        torch.cuda.synchronize()
        print(f"ceil_read slice {slice_wgs}", flush=True)
        j = rt.submit(k, (n_wg, 1, 1), args)
        if slice_wgs:
            rt.slice(j, slice_wgs)
        rt.schedule("fixed" if slice_wgs else "fifo", blocking=True, wait_done=True)
        rt.wait(j, 60_000_000_000)
        torch.cuda.synchronize()
    # thread t of workgroup w reads float4 number w * 256 * per + i * 256 + t
    s4 = src.cpu().view(n_wg, per, 256, 4).sum(dim=(1, 3)).reshape(-1)
    assert torch.equal(out.cpu(), s4)
