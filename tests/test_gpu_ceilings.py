"""GPU runs of the compute-ceiling probes (the FP32 FMA loop and the FP32
matrix-instruction loop the kernels' roofs are measured with): whole and
sliced with a ragged tail, every thread writes the value its chains or
accumulators reach, exactly (integers below 2^24 in FP32)."""
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
