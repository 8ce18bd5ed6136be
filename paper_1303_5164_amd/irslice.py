"""Slicing a kernel that knows nothing of slicing (Kernelet, Section 4.1).

The paper makes a compiled kernel sliceable by rewriting its PTX: the
workgroup index gains an offset, and the index of a multi-dimensional grid
is rebuilt from the linear one.  Here the same rewrite is done on the
AMDGPU LLVM IR of a kernel built in this repository (never on vendor
binaries): the HIP source is compiled for gfx950 to optimised device IR,
rewritten, and compiled to a code object that `kernelet_register_image`
loads.

The kernel must take one argument block by value (`__global__ void
k(Args a)`) and have every device function inlined into it (the usual
result of -O3).  The rewrite

  * appends a second by-value argument laid out as `kl_slice` (offset,
    count, gx, gy, gz, reserved), so the kernel takes (Args, kl_slice) like
    the source-level sliceable kernels;
  * computes at entry the linear index offset + workgroup_id.x of the 1-D
    slice launch, and from it, row-major over the original grid, the
    indices x = lin mod gx, y = (lin / gx) mod gy, z = lin / (gx gy);
  * replaces every read of the workgroup id (x, y, z) with those indices
    and every read of the grid's workgroup counts (gridDim, the first three
    implicit kernel arguments) with gx, gy, gz.

A kernel that reads the dispatch packet (its grid size in work-items) or
calls a non-inlined function that reads the workgroup id is rejected.  The
register use of the rewritten kernel is compared with the original's
(`resources`).

Usage: python -m paper_1303_5164_amd.irslice SOURCE.hip KERNEL [KERNEL ...] OUT.hsaco
       python -m paper_1303_5164_amd.irslice bench [INFLIGHT ...]   (matrix addition on the GPU)
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
LLVM = os.path.join(ROCM, "llvm", "bin")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "--cuda-device-only",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

SLICE_TYPE = "%kl.slice = type { i32, i32, i32, i32, i32, i32 }"


class SliceError(ValueError):
    pass


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise SliceError("command failed: " + " ".join(cmd) + "\n" + r.stdout[-4000:])
    return r.stdout


def device_ir(source: str, extra_flags=()) -> str:
    """Optimised gfx950 device IR (text) of a HIP source file."""
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.ll")
        _run(["hipcc", *HIP_FLAGS, *extra_flags, "-emit-llvm", "-S", source, "-o", out])
        return open(out).read()


def _matching_paren(s: str, i: int) -> int:
    depth = 0
    for j in range(i, len(s)):
        if s[j] == "(":
            depth += 1
        elif s[j] == ")":
            depth -= 1
            if depth == 0:
                return j
    raise SliceError("unbalanced parentheses in a definition")


def _split_top(s: str):
    """The comma-separated items of s at parenthesis depth 0."""
    out, depth, cur = [], 0, ""
    for ch in s:
        if ch == "(":
            depth += 1
        elif ch == ")":
            depth -= 1
        if ch == "," and depth == 0:
            out.append(cur.strip())
            cur = ""
        else:
            cur += ch
    if cur.strip():
        out.append(cur.strip())
    return out


def _functions(lines):
    """(name, first line, last line) of every function definition."""
    out, i = [], 0
    while i < len(lines):
        m = re.match(r"define .*?@([\w.$]+)\(", lines[i])
        if m:
            j = i
            while lines[j].rstrip() != "}":
                j += 1
            out.append((m.group(1), i, j))
            i = j
        i += 1
    return out


_WGID = re.compile(r"^(\s*)(%[\w.]+) = (?:tail |notail )?call (?:noundef )?i32 "
                   r"@llvm\.amdgcn\.workgroup\.id\.([xyz])\(\)")
_IMPL = re.compile(r"^\s*(%[\w.]+) = (?:tail )?call (?:noundef )?(?:nonnull )?"
                   r"(?:align \d+ )?ptr addrspace\(4\) @llvm\.amdgcn\.implicitarg\.ptr\(\)")
_GEP = re.compile(r"^\s*(%[\w.]+) = getelementptr (?:inbounds )?(?:nuw )?i8, ptr addrspace\(4\) "
                  r"(%[\w.]+), i64 (-?\d+)")
_LOAD = re.compile(r"^(\s*)(%[\w.]+) = load i32, ptr addrspace\(4\) (%[\w.]+)(,|$)")


def rewrite(ir: str, kernel: str) -> str:
    """The IR of `kernel` made sliceable (see the module docstring)."""
    lines = ir.split("\n")
    funcs = _functions(lines)
    kf = [f for f in funcs if f[0] == kernel]
    if not kf:
        raise SliceError(f"no definition of @{kernel}")
    _, k0, k1 = kf[0]
    if "amdgpu_kernel" not in lines[k0]:
        raise SliceError(f"@{kernel} is not a kernel")
    # other functions must not read the workgroup id (they would not see
    # the slice's offset)
    for name, a, b in funcs:
        if name == kernel or "amdgpu_kernel" in lines[a]:
            continue
        body = "\n".join(lines[a:b + 1])
        if "llvm.amdgcn.workgroup.id" in body or "llvm.amdgcn.implicitarg.ptr" in body:
            raise SliceError(f"@{name} reads the workgroup id or grid; inline it into "
                             f"@{kernel}")
    body = lines[k0 + 1:k1]
    if any("llvm.amdgcn.dispatch.ptr" in ln for ln in body):
        raise SliceError(f"@{kernel} reads the dispatch packet (grid size in work-items)")
    # slices are launched as 1-D workgroups of block_threads work-items, so a
    # kernel indexing its workgroup in y or z would see 0 there
    if any(re.search(r"@llvm\.amdgcn\.workitem\.id\.[yz]\(", ln) for ln in body):
        raise SliceError(f"@{kernel} uses a 2-D or 3-D workgroup (work-item id y or z); "
                         "slices run 1-D workgroups")

    # signature: exactly one by-value argument block, then the slice
    d = lines[k0]
    p0 = d.index("(", d.index("@" + kernel))
    p1 = _matching_paren(d, p0)
    params = _split_top(d[p0 + 1:p1])
    if len(params) != 1 or "byref(" not in params[0]:
        raise SliceError(f"@{kernel} must take exactly one argument block by value")
    lines[k0] = (d[:p1] + ", ptr addrspace(4) noundef readonly byref(%kl.slice) align 4 "
                 "%kl.s" + d[p1:])

    # reads of the workgroup id and of the grid's workgroup counts
    base = {}      # value -> byte offset into the implicit arguments
    for i in range(k0 + 1, k1):
        ln = lines[i]
        m = _WGID.match(ln)
        if m:
            lines[i] = f"{m.group(1)}{m.group(2)} = add i32 %kl.{m.group(3)}, 0"
            continue
        m = _IMPL.match(ln)
        if m:
            base[m.group(1)] = 0
            continue
        m = _GEP.match(ln)
        if m and m.group(2) in base:
            base[m.group(1)] = base[m.group(2)] + int(m.group(3))
            continue
        m = _LOAD.match(ln)
        if m and m.group(3) in base and base[m.group(3)] in (0, 4, 8):
            dim = "xyz"[base[m.group(3)] // 4]
            lines[i] = f"{m.group(1)}{m.group(2)} = add i32 %kl.g{dim}, 0"

    # every read of the grid's workgroup counts (the first 12 bytes of the
    # implicit arguments) must have become one of the rebuilt counts: a
    # vector, wider or unaligned read of them, or the pointer escaping,
    # would still see the 1-D slice launch
    for i in range(k0 + 1, k1):
        ln = lines[i]
        if _IMPL.match(ln):
            continue
        g = _GEP.match(ln)
        if g and g.group(2) in base:
            continue
        for v, off in base.items():
            if off < 12 and re.search(re.escape(v) + r"(?![\w.$])", ln):
                raise SliceError(f"@{kernel} reads the grid's workgroup counts in a form "
                                 f"the rewrite does not replace: {ln.strip()}")

    pre = ["  %kl.off = load i32, ptr addrspace(4) %kl.s, align 4",
           "  %kl.gxp = getelementptr inbounds i8, ptr addrspace(4) %kl.s, i64 8",
           "  %kl.gx = load i32, ptr addrspace(4) %kl.gxp, align 4",
           "  %kl.gyp = getelementptr inbounds i8, ptr addrspace(4) %kl.s, i64 12",
           "  %kl.gy = load i32, ptr addrspace(4) %kl.gyp, align 4",
           "  %kl.gzp = getelementptr inbounds i8, ptr addrspace(4) %kl.s, i64 16",
           "  %kl.gz = load i32, ptr addrspace(4) %kl.gzp, align 4",
           "  %kl.wg = call i32 @llvm.amdgcn.workgroup.id.x()",
           "  %kl.lin = add i32 %kl.off, %kl.wg",
           "  %kl.x = urem i32 %kl.lin, %kl.gx",
           "  %kl.q = udiv i32 %kl.lin, %kl.gx",
           "  %kl.y = urem i32 %kl.q, %kl.gy",
           "  %kl.z = udiv i32 %kl.q, %kl.gy"]
    # the entry block: right after the definition line, unless it opens
    # with a label
    at = k0 + 1
    if re.match(r"^[\w.]+:", lines[at]):
        at += 1
    lines[at:at] = pre
    out = "\n".join(lines)
    # the workgroup id x is read now; drop the hint that says it is not
    out = out.replace(' "amdgpu-no-workgroup-id-x"', "")
    if "declare noundef i32 @llvm.amdgcn.workgroup.id.x()" not in out and \
            "declare i32 @llvm.amdgcn.workgroup.id.x()" not in out:
        out += "\ndeclare i32 @llvm.amdgcn.workgroup.id.x()\n"
    # the slice type, after the module's other type definitions
    if SLICE_TYPE in out:
        return out
    m = list(re.finditer(r"^%[\w.]+ = type .*$", out, re.M))
    pos = m[-1].end() if m else out.index("\ndefine")
    return out[:pos] + "\n" + SLICE_TYPE + out[pos:]


def code_object(ir: str, out_path: str) -> str:
    """Compile device IR to a gfx950 code object at out_path."""
    with tempfile.TemporaryDirectory() as d:
        ll, obj = os.path.join(d, "k.ll"), os.path.join(d, "k.o")
        with open(ll, "w") as f:
            f.write(ir)
        _run([os.path.join(LLVM, "clang"), "-target", "amdgcn-amd-amdhsa", f"-mcpu={ARCH}",
              "-O3", "-c", ll, "-o", obj])
        _run([os.path.join(LLVM, "ld.lld"), "-shared", obj, "-o", out_path])
    return out_path


def resources(hsaco: str, kernel: str) -> dict:
    """Registers, LDS and kernel-argument bytes of `kernel` in a code
    object, from its metadata notes."""
    txt = _run([os.path.join(LLVM, "llvm-readelf"), "--notes", hsaco])
    i = txt.find(f".name:           {kernel}\n")
    if i < 0:
        i = txt.find(f".name: {kernel}")
    if i < 0:
        raise SliceError(f"no metadata for {kernel}")
    # the kernel's map runs from the previous '- .' entry start to the next
    start = txt.rfind("\n  - ", 0, i)
    end = txt.find("\n  - ", i)
    blk = txt[start:end if end > 0 else len(txt)]
    out = {}
    for key in ("vgpr_count", "sgpr_count", "agpr_count", "group_segment_fixed_size",
                "kernarg_segment_size", "private_segment_fixed_size"):
        m = re.search(r"\." + key + r":\s+(\d+)", blk)
        if m:
            out[key] = int(m.group(1))
    return out


def slice_source(source: str, kernels, out_path: str, extra_flags=()) -> dict:
    """Build one code object at out_path holding the sliceable versions of
    `kernels` (a name or a list) of a HIP source; returns, per kernel, the
    resources of the original and of the rewritten kernel."""
    kernels = [kernels] if isinstance(kernels, str) else list(kernels)
    ir = device_ir(source, extra_flags)
    info = {}
    with tempfile.TemporaryDirectory() as d:
        orig = code_object(ir, os.path.join(d, "orig.hsaco"))
        for k in kernels:
            info[k] = {"original": resources(orig, k)}
    rw = ir
    for k in kernels:
        rw = rewrite(rw, k)
    code_object(rw, out_path)
    for k in kernels:
        info[k]["sliced"] = resources(out_path, k)
    return info


def bench(n: int = 8192, reps: int = 5, inflight: int = 2) -> dict:
    """The paper's matrix addition (n x n, fp32) through the sliceable code
    object on the GPU: time of the whole grid in one launch and in slices of
    b * n_cu workgroups, against torch's own elementwise addition of the
    same arrays (a reference for a plain, unsliced kernel)."""
    import ctypes as C
    import statistics
    import time

    import torch

    import paper_1303_5164_amd as K
    from . import build as B

    class Args(C.Structure):
        _fields_ = [("a", C.c_void_p), ("b", C.c_void_p), ("c", C.c_void_p),
                    ("n", C.c_uint32)]

    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(0)
    a = torch.rand(n * n, device=dev, generator=g)
    b = torch.rand(n * n, device=dev, generator=g)
    c = torch.empty_like(a)
    ref = a + b
    args = Args(a.data_ptr(), b.data_ptr(), c.data_ptr(), n)
    nb = (n + 15) // 16
    with open(B.PLAIN_IMAGE, "rb") as f:
        image = f.read()
    out = {"n": n, "workgroups": nb * nb, "bytes": 12 * n * n, "inflight": inflight,
           "runs": []}
    with K.Runtime(0, inflight=inflight) as rt:
        k = rt.register_image("plain_matadd", image, "kl_plain_matadd", C.sizeof(Args))
        n_cu = rt.cfg.n_cu

        def once(slice_wgs):
            c.zero_()
            torch.cuda.synchronize()
            j = rt.submit(k, (nb, nb, 1), args)
            if slice_wgs:
                rt.slice(j, slice_wgs)
            t0 = time.perf_counter()
            rt.schedule("fixed" if slice_wgs else "fifo", blocking=True, wait_done=True)
            t = time.perf_counter() - t0
            rt.reap()
            assert torch.equal(c, ref)
            return t

        def run(slice_wgs):
            # wall time of a schedule call with no timing events, then one
            # more run whose launches carry events: the GPU time of its slices
            ts = [once(slice_wgs) for _ in range(reps + 1)]
            rt.time_kernel(k, True)
            once(slice_wgs)
            ms, nl, _ = rt.kernel_time(k)
            rt.time_kernel(k, False)
            return statistics.median(ts[1:]), ms, nl

        t_whole, g_whole, _ = run(0)
        out["runs"].append({"slice_wgs": 0, "ms": t_whole * 1e3, "gpu_ms": g_whole})
        b_ = 1
        while b_ * n_cu < nb * nb:
            t, gms, nl = run(b_ * n_cu)
            out["runs"].append({"slice_wgs": b_ * n_cu, "launches": nl, "ms": t * 1e3,
                                "gpu_ms": gms, "overhead": t / t_whole - 1.0})
            b_ *= 2
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.add(a, b, out=c)
    ev[0].record()
    for _ in range(reps):
        torch.add(a, b, out=c)
    ev[1].record()
    torch.cuda.synchronize()
    out["torch_add_ms"] = ev[0].elapsed_time(ev[1]) / reps
    return out


def main():
    if len(sys.argv) >= 2 and sys.argv[1] == "bench":
        import json
        res = [bench(inflight=int(x)) for x in (sys.argv[2:] or ["2"])]
        print(json.dumps(res, indent=1))
        return
    if len(sys.argv) < 4:
        print(__doc__, file=sys.stderr)
        sys.exit(2)
    info = slice_source(sys.argv[1], sys.argv[2:-1], sys.argv[-1])
    for k, v in info.items():
        print(k, v)


if __name__ == "__main__":
    main()
