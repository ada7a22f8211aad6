"""The C-ABI library loads without a GPU, exports every declared symbol, and
serves a plain C program (host-side calls)."""
import os
import re

import numpy as np
import pytest

from paper_2510_23446_amd import tcf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(tcf\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    L = tcf.lib()
    names = declared_functions()
    assert "tcf_create" in names and "tcf_step" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/ but not exported"
    assert set(tcf.EXPORTS) <= set(names)


def test_default_options_and_error_string():
    o = tcf.default_options()
    assert o.precision == tcf.TCF_FP64 and o.pcg_rtol == 1e-10
    assert isinstance(tcf.lib().tcf_last_error(None), bytes)


def test_c_program_uses_the_abi_without_a_gpu(tmp_path):
    """A plain C program includes tcf.h, links libtcf.so, describes the
    2x2x2-patch cube and creates the handle (host work only): its topology
    counts and footprints equal the binding's, and the error paths return
    the documented codes."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_2510_23446_amd")
    exe = str(tmp_path / "c_abi_host")
    cmd = [gcc, "-std=c99", "-O1", os.path.join(root, "tests", "c_abi_host.c"),
           "-I", os.path.join(root, "include"), "-L", pkg, "-ltcf", "-lm",
           "-Wl,-rpath," + pkg, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = dict(l.split(" ", 1) for l in r.stdout.strip().splitlines())
    import workloads as W
    from paper_2510_23446_amd import tcf
    p = tcf.Problem(W.plain_fp64())
    want = [int(v) for v in p.tcf_get_topology(tcf.TCF_TOPO_COUNTS)]
    assert [int(v) for v in lines["counts"].split()] == want
    b64, b32 = p.tcf_footprint()
    assert [int(v) for v in lines["footprint"].split()] == [b64, b32]
    assert int(lines["step_before_setup"]) == tcf.TCF_ESTATE
    assert lines["negative_sigma"].split() == [str(tcf.TCF_EINVAL), "null"]


def _vm_size_mib():
    with open("/proc/self/status") as f:
        for line in f:
            if line.startswith("VmSize"):
                return int(line.split()[1]) / 1024.0
    pytest.skip("no /proc/self/status")


def test_server_lifecycle_without_a_device():
    """With no HIP device every request fails at its worker's first HIP call.
    The server must still admit, fail and count each one with a message, and
    join finished workers as it goes: before that fix every finished worker
    kept its thread stack (about 8 MiB of address space) until the server was
    destroyed."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("checks the host-side path taken when no device is present")
    import workloads as W

    prob = W.plain_fp64().with_steps(1)
    srv = tcf.Server(max_bytes=64 << 30, max_slots=4)
    try:
        first = [srv.tcf_server_submit(prob) for _ in range(32)]
        assert all(srv.tcf_server_wait(i) == tcf.TCF_EHIP for i in first)
        # a leak grows with every batch; a one-off reservation (a new malloc
        # arena reserves 64 MiB of address space) shows in one batch only, so
        # of four batches all but the largest together stay under 64 MiB (a
        # kept thread stack per request would add about 1 GiB per batch)
        grown = []
        for _ in range(4):
            v0 = _vm_size_mib()
            more = [srv.tcf_server_submit(prob) for _ in range(128)]
            assert all(srv.tcf_server_wait(i) == tcf.TCF_EHIP for i in more)
            grown.append(_vm_size_mib() - v0)
        assert sum(sorted(grown)[:-1]) < 64.0, \
            f"address space grew by {grown} MiB over four batches of 128"
        assert "hipStreamCreateWithFlags" in srv.tcf_server_error(more[-1])
        assert srv.tcf_server_poll(more[0]) == tcf.TCF_REQ_FAILED
        # a rejected description gets no id and leaves the other requests'
        # callbacks in place
        bad = W.plain_fp64().with_steps(1)
        bad.sigma = -np.ones_like(np.asarray(bad.sigma, dtype=float))
        with pytest.raises(tcf.TcfError) as err:
            srv.tcf_server_submit(bad)
        assert err.value.code == tcf.TCF_EINVAL
        assert srv._keep[first[0]][3] is prob and len(srv._keep) == 32 + 4 * 128
        st = srv.tcf_server_stats()
        assert st["submitted"] == st["admitted"] == st["failed"] == 32 + 4 * 128
        assert st["completed"] == st["running"] == st["queued"] == 0
    finally:
        srv.tcf_server_destroy()


def test_server_rejects_an_oversize_request_without_a_device():
    """Admission by footprint is host work: a request larger than the budget
    is refused with TCF_ENOMEM at submission, keeps an id of its own (so the
    ids of later requests stay consistent) and does not block the queue."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("checks the host-side path taken when no device is present")
    import workloads as W

    prob = W.plain_fp64().with_steps(1)
    fp = tcf.Problem(prob).tcf_footprint()[0]
    srv = tcf.Server(max_bytes=fp // 2, max_slots=2)
    try:
        with pytest.raises(tcf.TcfError) as err:
            srv.tcf_server_submit(prob, precision="fp64")
        assert err.value.code == tcf.TCF_ENOMEM
        small = W.plain_fp64().with_steps(1)
        small.nel = [np.minimum(np.asarray(v), 2).astype(np.int32) for v in small.nel]
        assert tcf.Problem(small).tcf_footprint()[0] <= fp // 2
        i = srv.tcf_server_submit(small, precision="fp64")
        assert i == 1  # id 0 is the rejected request
        assert srv.tcf_server_poll(0) == tcf.TCF_REQ_FAILED
        assert "budget" in srv.tcf_server_error(0)
        assert srv.tcf_server_wait(i) == tcf.TCF_EHIP
    finally:
        srv.tcf_server_destroy()


def test_server_concurrent_submissions_without_a_device():
    """Four threads submit 16 requests each at once (ctypes releases the
    GIL, so the submissions race inside the library): the ids are exactly
    0..63, each once, and every request ends failed at its worker's first
    HIP call with that call named."""
    import threading

    import torch

    if torch.cuda.is_available():
        pytest.skip("checks the host-side path taken when no device is present")
    import workloads as W

    prob = W.plain_fp64().with_steps(1)
    srv = tcf.Server(max_bytes=64 << 30, max_slots=4)
    ids, errs = [], []

    def submit():
        try:
            for _ in range(16):
                ids.append(srv.tcf_server_submit(prob))
        except Exception as e:  # reported below
            errs.append(e)

    try:
        threads = [threading.Thread(target=submit) for _ in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        assert not errs, errs
        assert sorted(ids) == list(range(64))
        assert all(srv.tcf_server_wait(i) == tcf.TCF_EHIP for i in ids)
        assert all(srv.tcf_server_poll(i) == tcf.TCF_REQ_FAILED for i in ids)
        assert "hipStreamCreateWithFlags" in srv.tcf_server_error(ids[-1])
    finally:
        srv.tcf_server_destroy()


def test_marker_ranges_are_linked():
    """Setup, steps, PCG solves and refinement sweeps open named ranges on
    the ROCm marker timeline: the library imports the marker API."""
    import subprocess
    so = os.path.join(ROOT, "paper_2510_23446_amd", "libtcf.so")
    out = subprocess.run(["nm", "-D", "--undefined-only", so], capture_output=True, text=True,
                         check=True).stdout
    assert "roctxRangePushA" in out and "roctxRangePop" in out
    src = open(os.path.join(ROOT, "paper_2510_23446_amd", "csrc", "tcf_api.hip")).read()
    for name in ("tcf setup", "tcf step: one time step", "PCG solve", "refinement sweep"):
        assert f'Range rg("{name}")' in src or f'("{name}' in src, name
