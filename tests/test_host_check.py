"""Host-memory checks of the C-ABI: pf_host_check (built with the library) calls
every entry point with exactly sized heap arrays, ragged sizes and invalid
arguments against the host engine compiled under AddressSanitizer, with leak
detection on (leaks inside the HIP runtime's own frames are suppressed).  On
the CPU it runs the calls that need no device; on the GPU it also drives
handles of every integrator, adaptive runs, checkpoints, sparse storage and a
batch."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2601_16522_amd", "pf_host_check")


def _run(mode, tmp_path):
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is not built; run paper_2601_16522_amd/build.py")
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\nleak:libdrm\n")
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               LSAN_OPTIONS=f"suppressions={supp}:print_suppressions=0")
    p = subprocess.run([EXE, mode], capture_output=True, text=True, timeout=600, env=env)
    print(p.stdout[-3000:], p.stderr[-6000:], flush=True)
    assert p.returncode == 0, (p.returncode, p.stderr[-3000:])
    assert "AddressSanitizer" not in p.stderr and "LeakSanitizer" not in p.stderr
    assert p.stdout.strip().endswith("ok")
    return p.stdout


def test_host_calls_under_asan(tmp_path):
    out = _run("host", tmp_path)
    assert "host error norms: 224 shapes" in out


@pytest.mark.gpu
def test_device_calls_under_asan(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = _run("gpu", tmp_path)
    assert "batch of 3: ok" in out
