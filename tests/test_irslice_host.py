"""The IR slicer on the CPU (Section 4.1: a compiled kernel made sliceable
by rewriting it): the rewritten device IR of kernels written without
slicing takes (Args, kl_slice), reads the workgroup id only to rebuild the
original grid's indices, compiles to a gfx950 code object with the kernel
argument layout the runtime passes, and kernels the rewrite cannot serve
are refused.  No GPU calls."""
import os
import re

import pytest

from paper_1303_5164_amd import build as B
from paper_1303_5164_amd import irslice as I

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ir():
    return I.device_ir(B.PLAIN_SOURCE)


def _body(text, kernel):
    lines = text.split("\n")
    for name, a, b in I._functions(lines):
        if name == kernel:
            return lines[a], "\n".join(lines[a + 1:b])
    raise AssertionError(kernel)


@pytest.mark.parametrize("kernel", B.PLAIN_KERNELS)
def test_rewrite_replaces_every_index_read(ir, kernel):
    head0, body0 = _body(ir, kernel)
    out = I.rewrite(ir, kernel)
    head, body = _body(out, kernel)
    assert head.count("byref(") == 2 and "byref(%kl.slice) align 4 %kl.s)" in head
    assert I.SLICE_TYPE in out
    # the only workgroup-id read left is the slice launch's own, at entry
    assert len(re.findall(r"@llvm\.amdgcn\.workgroup\.id\.", body)) == 1
    assert "%kl.wg = call i32 @llvm.amdgcn.workgroup.id.x()" in body
    # every original read became one of the rebuilt indices or counts
    n_ids = len(re.findall(r"call (?:noundef )?i32 @llvm\.amdgcn\.workgroup\.id\.", body0))
    assert len(re.findall(r"= add i32 %kl\.[xyz], 0", body)) == n_ids
    if kernel == "kl_plain_visit3d":
        # gridDim.x, .y, .z: the first three implicit arguments
        assert len(re.findall(r"= add i32 %kl\.g[xyz], 0", body)) == 3
    # other kernels of the module are untouched
    other = [k for k in B.PLAIN_KERNELS if k != kernel][0]
    assert _body(out, other) == _body(ir, other)


def test_code_object_layout_and_registers(tmp_path):
    info = I.slice_source(B.PLAIN_SOURCE, B.PLAIN_KERNELS, str(tmp_path / "k.hsaco"))
    m, v = info["kl_plain_matadd"], info["kl_plain_visit3d"]
    # (Args, kl_slice): 32-byte argument block, then 24 bytes of slice
    assert m["original"]["kernarg_segment_size"] == 32
    assert m["sliced"]["kernarg_segment_size"] == 32 + 24
    # the original read gridDim through the implicit arguments; the sliced
    # kernel reads the slice block instead and needs none
    assert v["original"]["kernarg_segment_size"] > 24 + 24
    assert v["sliced"]["kernarg_segment_size"] == 24 + 24
    for k in info.values():
        assert k["sliced"]["vgpr_count"] <= k["original"]["vgpr_count"] + 4
        assert k["sliced"]["private_segment_fixed_size"] == 0
        assert k["sliced"]["group_segment_fixed_size"] == k["original"]["group_segment_fixed_size"]


def _write(tmp_path, src):
    p = tmp_path / "k.hip"
    p.write_text("#include <hip/hip_runtime.h>\n#include <stdint.h>\n"
                 "struct A { uint32_t* o; uint32_t n; };\n" + src)
    return str(p)


def test_refuses_what_it_cannot_rewrite(tmp_path):
    cases = {
        "noinline": """
__device__ __attribute__((noinline)) uint32_t which() { return blockIdx.y; }
extern "C" __global__ void k(A a) { a.o[threadIdx.x] = which(); }
""",
        "two_args": """
extern "C" __global__ void k(A a, uint32_t extra) { a.o[blockIdx.x] = extra; }
""",
        "scalar_first": """
extern "C" __global__ void k(uint32_t extra, A a) { a.o[blockIdx.x] = extra; }
""",
        "no_block": """
extern "C" __global__ void k(uint32_t* o) { o[blockIdx.x] = 1; }
""",
        "dispatch": """
extern "C" __global__ void k(A a) {
    const uint32_t* p = (const uint32_t*)__builtin_amdgcn_dispatch_ptr();
    a.o[blockIdx.x] = p[3];
}
""",
    }
    for name, src in cases.items():
        ir = I.device_ir(_write(tmp_path, src))
        with pytest.raises(I.SliceError):
            I.rewrite(ir, "k")
    with pytest.raises(I.SliceError):
        I.rewrite(I.device_ir(B.PLAIN_SOURCE), "no_such_kernel")


def test_refuses_two_dimensional_workgroups(tmp_path):
    """The paper's matrix addition with 16 x 16 workgroups reads threadIdx.y;
    slices run 1-D workgroups, so the rewrite refuses it."""
    src = """
extern "C" __global__ void k(A a) {
    uint32_t x = blockIdx.x * 16 + threadIdx.x, y = blockIdx.y * 16 + threadIdx.y;
    if (x < a.n && y < a.n) a.o[y * a.n + x] = 1;
}
"""
    with pytest.raises(I.SliceError, match="work-item id"):
        I.rewrite(I.device_ir(_write(tmp_path, src)), "k")


# A kernel whose two workgroup counts are read by one <2 x i32> load of the
# implicit arguments (hand-written IR: the vectoriser may or may not merge
# such reads in compiled code).
_VEC_GRID_IR = """
%struct.A = type { ptr, i32 }

define amdgpu_kernel void @k(ptr addrspace(4) noundef readonly byref(%struct.A) align 8 %0) {
  %impl = tail call ptr addrspace(4) @llvm.amdgcn.implicitarg.ptr()
  %g = load <2 x i32>, ptr addrspace(4) %impl, align 4
  %gx = extractelement <2 x i32> %g, i64 0
  %op = load ptr, ptr addrspace(4) %0, align 8
  store i32 %gx, ptr %op, align 4
  ret void
}

declare ptr addrspace(4) @llvm.amdgcn.implicitarg.ptr()
"""


def test_refuses_merged_grid_reads():
    with pytest.raises(I.SliceError, match="workgroup counts"):
        I.rewrite(_VEC_GRID_IR, "k")
    # the same read as one i32 per count is rewritten
    ok = _VEC_GRID_IR.replace(
        "%g = load <2 x i32>, ptr addrspace(4) %impl, align 4\n"
        "  %gx = extractelement <2 x i32> %g, i64 0",
        "%gx = load i32, ptr addrspace(4) %impl, align 4")
    out = I.rewrite(ok, "k")
    assert "%gx = add i32 %kl.gx, 0" in out


def test_built_image_exists():
    """build() leaves the sliceable code object beside the library."""
    assert os.path.exists(B.PLAIN_IMAGE) and os.path.getsize(B.PLAIN_IMAGE) > 1000
