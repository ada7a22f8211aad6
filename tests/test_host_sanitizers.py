"""Host code under sanitizers: the topology code and the loop-split host
plan, built with g++ (host only, no GPU code) with AddressSanitizer and
UBSan, run on four layouts."""
import os

import pytest


def test_topology_code_is_clean_under_sanitizers(tmp_path):
    """The host topology code and the loop-split host plan (loop rows, psi,
    per-patch plan), built with AddressSanitizer and UBSan (any finding aborts), run on four
    layouts (a floating conductor and two checkerboards among them) without
    a report."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "topology_sanitize")
    cmd = [gxx, "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(root, "include"),
           os.path.join(root, "tests", "topology_sanitize.cpp"),
           os.path.join(root, "paper_2510_23446_amd", "csrc", "tcf_topology.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="verify_asan_link_order=0")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    lines = r.stdout.strip().splitlines()
    assert len(lines) == 4
    for line in lines:
        f = line.split()
        assert int(f[f.index("loop") + 2]) > 0 and int(f[f.index("psi") + 2]) > 0, line
        assert int(f[f.index("plan") + 2]) > 0, line
        assert line.endswith("err ''"), line
