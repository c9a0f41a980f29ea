"""The library's host code (planners, schedules, group and chunk bookkeeping,
argument checks) under AddressSanitizer and ThreadSanitizer, on the CPU.

The host sources are compiled with g++ -fsanitize=address against a test
double of the HIP runtime (tests/hostsim: device memory is host memory, no
kernel runs), then driven through the Python binding in a child process with
the sanitizer preloaded: every create / upload / assemble / pipelined
assemble / apply / solver path for several shapes and options, and the error
paths.  Any out-of-bounds or use-after-free access in host code fails the
test.  Nothing numeric is checked here (no kernel runs); the GPU tests do that.
"""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_08382_amd", "csrc")
HOSTSIM = os.path.join(ROOT, "tests", "hostsim")
SOURCES = ["context.cpp", "solver.cpp", "host_api.cpp", "host_sparse.cpp"]


def _libasan():
    try:
        p = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _build_hostsim(out, sanitizer):
    """The library's host sources + the runtime test double + stubbed
    launchers, built with g++ -fsanitize=<sanitizer>."""
    # every kernel launcher declared in the two launcher headers returns
    # success without running anything
    stubs = ['#include "kernels.hpp"', '#include "solver_kernels.hpp"', "namespace fetif {"]
    for h in ("kernels.hpp", "solver_kernels.hpp"):
        with open(os.path.join(CSRC, h)) as f:
            text = f.read()
        for m in re.finditer(r"hipError_t\s+(launch_\w+)\s*\(([^;]*?)\);", text, re.S):
            check = "hostsim_check_stream(st); " if re.search(r"hipStream_t\s+st\b", m.group(2)) else ""
            # the debug scan reports "nothing found" (its sentinel) in host memory
            extra = "*first = ~0ull; " if m.group(1) == "launch_first_nonfinite" else ""
            stubs.append(f"hipError_t {m.group(1)}({m.group(2)}) {{ {check}{extra}return hipSuccess; }}")
    # the static scratch of the allocation-free apply: host memory here
    stubs.append("hipError_t static_scratch_address(int, void** out) "
                 "{ static unsigned char* buf = new unsigned char[kStaticScratchBytes]; *out = buf; return hipSuccess; }")
    stubs.append("}")
    stub_cpp = out / "launch_stubs.cpp"
    stub_cpp.write_text("\n".join(stubs) + "\n")
    lib = out / f"libfetiF_hostsim_{sanitizer}.so"
    cmd = (["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", f"-fsanitize={sanitizer}", "-fno-omit-frame-pointer",
            "-I" + HOSTSIM, "-I" + CSRC, os.path.join(HOSTSIM, "runtime_stand_in.cpp"), str(stub_cpp)]
           + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", str(lib), "-lpthread"])
    subprocess.run(cmd, check=True)
    return str(lib)


def _libtsan():
    try:
        p = subprocess.run(["g++", "-print-file-name=libtsan.so"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def hostsim_lib(tmp_path_factory):
    if shutil.which("g++") is None or _libasan() is None:
        pytest.skip("g++ with AddressSanitizer is not available")
    return _build_hostsim(tmp_path_factory.mktemp("hostsim"), "address")


@pytest.fixture(scope="module")
def hostsim_tsan_lib(tmp_path_factory):
    if shutil.which("g++") is None or _libtsan() is None:
        pytest.skip("g++ with ThreadSanitizer is not available")
    return _build_hostsim(tmp_path_factory.mktemp("hostsim_tsan"), "thread")


DRIVER = r'''
import sys
import numpy as np
sys.path.insert(0, ROOT)
from paper_2502_08382_amd.fetif import load_library, FetiContext, FetiError
from paper_2502_08382_amd import subdomain_dict, values_in_pattern
from synth import config_problem, make_problem
load_library(LIB)
ST = 0x7f0012345670           # any 64-bit stream handle: the test double ignores it


def expect(status, fn):
    try:
        fn()
    except FetiError as e:
        assert e.status == status, (e.status, str(e))
        return
    raise AssertionError("expected status %d" % status)


def flow(prob, with_elements=False, **opts):
    subs = [subdomain_dict(s, with_elements) for s in prob.subs]
    kv = [s.Kreg.data for s in prob.subs]
    ctx = FetiContext(subs, prob.n_lambda, device=0, **opts)
    info = ctx.info()
    assert 1 <= info["assembly_groups"] <= min(prob.nsub, opts.get("assembly_groups", 1))
    assert info["nsub"] == prob.nsub and info["n_lambda"] == prob.n_lambda
    assert info["sum_m"] == sum(s.m for s in prob.subs)
    assert info["f_tri_elements"] == sum(s.m * (s.m + 1) // 2 for s in prob.subs)
    assert info["apply_elements"] >= info["f_tri_elements"] and info["trsm_levels"] > 0
    expect(3, lambda: ctx.assemble(stream=ST))            # before any upload
    ctx.factor_upload(kv, stream=ST)
    ctx.assemble(stream=ST)
    for panel, chunk in ((16, 16), (48, 64), (96, 32)):
        ctx.set_assembly(panel, chunk)
        ctx.assemble(stream=ST)
        ctx.factor_assemble(kv, stream=ST)
    # the TRSM path (backward solve + SpMM), re-planned with the panel width
    ctx.set_assembly_path(1)
    ctx.assemble(stream=ST)
    expect(6, lambda: ctx.factor_assemble(kv, stream=ST))
    ctx.set_assembly(32, 0)
    ctx.assemble(stream=ST)
    ctx.set_assembly_path(0)
    ctx.set_assembly(96, 32)
    ctx.assemble(stream=ST)
    n = prob.n_lambda
    lam = np.zeros(n)
    q = np.zeros(n)
    for seg in ((0, 2, 3, 4, 8) if max(s.m for s in prob.subs) <= 4096 else (2, 4, 8)):
        for split in (0, 1):
            for band in (1, 3000, 0):
                ctx.set_apply(band, 2, 1, split, seg)
                ctx.apply(lam.ctypes.data, q.ctypes.data, stream=ST)
                try:
                    ctx.apply_static(lam.ctypes.data, q.ctypes.data, stream=ST)
                except FetiError as e:   # partials beyond the static scratch
                    assert e.status == 6 and "static scratch" in str(e), str(e)
    ctx.apply_implicit(lam.ctypes.data, q.ctypes.data, stream=ST)
    for sg in (0, 1, 0):
        ctx.apply_host(lam, q, cpu_scatter_gather=sg, stream=ST)
    f = np.zeros(sum(s.n for s in prob.subs))
    e = np.zeros(sum(s.R.shape[1] for s in prob.subs))
    d = np.zeros(n)
    ctx.coarse_rhs(f.ctypes.data, e.ctypes.data, stream=ST)
    ctx.dual_rhs(f.ctypes.data, d.ctypes.data, stream=ST)
    ctx.pcpg(d.ctypes.data, e.ctypes.data, lam.ctypes.data, fixed_iters=3, use_graph=True, stream=ST)
    ctx.pcpg(d.ctypes.data, e.ctypes.data, lam.ctypes.data, fixed_iters=2, precond=1, stream=ST)
    ctx.pcpg(d.ctypes.data, e.ctypes.data, lam.ctypes.data, fixed_iters=2, precond=2, use_graph=True, stream=ST)
    ctx.precond_values([values_in_pattern(s.K, s.Kreg) for s in prob.subs[:2]], first=0)
    ctx.pcpg(d.ctypes.data, e.ctypes.data, lam.ctypes.data, fixed_iters=2, precond=2, stream=ST)
    if with_elements:
        ne = sum(len(s.theta) for s in prob.subs)
        dth = np.zeros(ne)
        ctx.apply_backward(lam.ctypes.data, lam.ctypes.data, q.ctypes.data, dth.ctypes.data, stream=ST)
    for i in range(prob.nsub):
        ctx.download_F(i)
    # a non-SPD K_reg in the last subdomain: nothing counts as uploaded after it
    bad = [v.copy() for v in kv]
    A = prob.subs[-1].Kreg.tocoo()
    bad[-1][np.nonzero(A.row == A.col)[0][2]] = -1.0
    expect(5, lambda: ctx.factor_assemble(bad, stream=ST))
    expect(3, lambda: ctx.apply(lam.ctypes.data, q.ctypes.data, stream=ST))
    expect(3, lambda: ctx.apply_static(lam.ctypes.data, q.ctypes.data, stream=ST))
    expect(5, lambda: ctx.factor_upload(bad, stream=ST))
    ctx.factor_upload(kv, stream=ST)
    ctx.assemble(stream=ST)
    ctx.close()


flow(config_problem(1), with_elements=True)
flow(make_problem(1, "heat", [[7]], 0.0, dirichlet_axis=0, seed=1), with_elements=True)
flow(make_problem(1, "heat", [[5, 5, 12]], 0.0, dirichlet_axis=0, seed=1), assembly_groups=2, nthreads=1)
flow(config_problem(5, scale=(2, 5)), with_elements=True, assembly_groups=3, nthreads=2, debug_checks=1)
flow(config_problem(2, scale=(3, 6), elem="simplex"), assembly_groups=8, nthreads=1, f_storage="f32")
flow(make_problem(3, "elasticity", [[3, 4, 2], [3, 2], [2, 3]], 0.3, dirichlet_axis=2, seed=3),
     assembly_groups=5, nthreads=2, f_storage="bf16")
flow(make_problem(2, "heat", [[7, 13, 5], [9, 11]], 0.5, dirichlet_axis=0, seed=9), assembly_groups=100)
# the Schur-complement order (multiplier nodes last)
flow(config_problem(2, scale=(2, 6)), schur_order=1, assembly_groups=2)
flow(make_problem(3, "elasticity", [[3, 4], [3, 2], [2, 3]], 0.3, dirichlet_axis=2, seed=3), schur_order=1,
     f_storage="bf16")
# more than 4096 multipliers in a subdomain (flat slabs, m = 8450 and 4225):
# the segmented apply serves it, the whole-row kernel is refused
wide = make_problem(3, "heat", [[64], [64], [2, 2]], 0.0, dirichlet_axis=2, seed=1)
assert max(s.m for s in wide.subs) > 8192
flow(wide)
wctx = FetiContext([subdomain_dict(s) for s in wide.subs], wide.n_lambda, device=0)
expect(6, lambda: wctx.set_apply(0, 2, 1, 0, 0))
wctx.set_apply(3000, 2, 1, 1, 8)
wctx.close()
print("hostsim flows done")
'''


def test_host_code_under_address_sanitizer(hostsim_lib):
    env = dict(os.environ)
    env["LD_PRELOAD"] = _libasan()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["HOSTSIM_STREAM"] = "0x7f0012345670"    # the stream handle the driver passes (ST)
    code = f"ROOT = {ROOT!r}\nLIB = {hostsim_lib!r}\n" + DRIVER
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    out = p.stdout + p.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert p.returncode == 0, out[-4000:]
    assert "hostsim flows done" in p.stdout


TRUNCATION = r'''
import ctypes, sys
sys.path.insert(0, ROOT)
from paper_2502_08382_amd.fetif import load_library, FetiContext
from paper_2502_08382_amd import subdomain_dict
from synth import config_problem
load_library(LIB)
ST = 0x7f0012345670
prob = config_problem(1)
ctx = FetiContext([subdomain_dict(s) for s in prob.subs], prob.n_lambda, device=0)
ctx.factor_upload([s.Kreg.data for s in prob.subs], stream=ST)
ctx.assemble(stream=ST)                       # declared argument types: the handle arrives whole
print("declared binding ok", flush=True)
raw = ctypes.CDLL(LIB).fetiF_assemble         # the same entry point without declared argument types
raw(ctypes.c_void_p(ctx.h.value), ST)         # ctypes passes the int as a C int: 32 bits
print("not reached", flush=True)
'''


def test_stream_handle_cut_to_32_bits_is_caught(hostsim_lib):
    """A failure mode that would crash a GPU run: a binding without
    declared argument types hands a 64-bit stream handle to the library as
    a C int, and the runtime receives another value.  With
    the declared types the handle arrives whole; through an undeclared
    ctypes function the test double of the runtime sees the cut handle and
    aborts (on the GPU the runtime would dereference it)."""
    env = dict(os.environ)
    env["LD_PRELOAD"] = _libasan()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:handle_abort=0"
    env["HOSTSIM_STREAM"] = "0x7f0012345670"
    code = f"ROOT = {ROOT!r}\nLIB = {hostsim_lib!r}\n" + TRUNCATION
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert "declared binding ok" in p.stdout, p.stdout + p.stderr[-3000:]
    assert "not reached" not in p.stdout
    assert p.returncode != 0 and "reached the runtime, expected 0x7f0012345670" in p.stderr, p.stderr[-3000:]


PIPELINE = r'''
import sys
sys.path.insert(0, ROOT)
from paper_2502_08382_amd.fetif import load_library, FetiContext
from paper_2502_08382_amd import subdomain_dict
from synth import config_problem
load_library(LIB)
ST = 0x7f0012345670
prob = config_problem(2, scale=SCALE)
kv = [s.Kreg.data for s in prob.subs]
ctx = FetiContext([subdomain_dict(s) for s in prob.subs], prob.n_lambda, device=0, assembly_groups=8, nthreads=16)
assert ctx.info()["assembly_groups"] == 8
ctx.factor_upload(kv, stream=ST)
ctx.factor_assemble(kv, stream=ST)
ctx.factor_upload(kv[7:107], first=7, stream=ST)
ctx.factor_assemble(kv, stream=ST)
ctx.assemble(stream=ST)
ctx.close()
print("pipeline done", flush=True)
'''


def _run_pipeline(lib, preload, options_var, options, scale):
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    env[options_var] = options
    env["HOSTSIM_STREAM"] = "0x7f0012345670"
    code = f"ROOT = {ROOT!r}\nLIB = {lib!r}\nSCALE = {scale!r}\n" + PIPELINE
    return subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)


def test_full_size_pipelined_preprocessing_under_address_sanitizer(hostsim_lib):
    """The benchmark's pipelined leg on the host side at full size: the
    512-subdomain heat workload (12^3 hexes), 8 assembly groups, 16 host
    threads, factor upload then pipelined factorisation + copy + assembly
    (twice, with a partial upload between), under AddressSanitizer."""
    p = _run_pipeline(hostsim_lib, _libasan(), "ASAN_OPTIONS", "detect_leaks=0:abort_on_error=0", None)
    out = p.stdout + p.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert p.returncode == 0 and "pipeline done" in p.stdout, out[-4000:]


def test_pipelined_preprocessing_under_thread_sanitizer(hostsim_tsan_lib):
    """The same flow under ThreadSanitizer (data races between the host
    threads of the factorisation, the chunk and group bookkeeping and the
    staging writes): 512 subdomains of 6^3 hexes, 8 groups, 16 threads."""
    p = _run_pipeline(hostsim_tsan_lib, _libtsan(), "TSAN_OPTIONS", "halt_on_error=1 report_signal_unsafe=0", (8, 6))
    out = p.stdout + p.stderr
    assert "ThreadSanitizer" not in out, out[-4000:]
    assert p.returncode == 0 and "pipeline done" in p.stdout, out[-4000:]
