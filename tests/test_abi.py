"""The C-ABI library loads without a GPU and exports every symbol the header
declares; host-only calls answer.  No compute call is made here."""
import ctypes as C
import os
import re

import pytest

import paper_2601_16522_amd as pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported():
    names = _declared()
    assert len(names) >= 20
    L = C.CDLL(pf.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(pf.EXPORTS) == names


def test_supported_nphi_and_errors_without_device():
    assert pf.supported_nphi() == [2, 3, 4, 8, 9, 13]
    L = pf.lib()
    assert L.pf_create(None, None) == -1          # PF_EINVAL before any device work
    assert L.pf_last_error(None) == b"null handle"


def test_binding_fails_loudly_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(pf, "LIB_PATH", str(tmp_path / "libpf.so"))
    monkeypatch.setattr(pf, "_lib", None)
    with pytest.raises(ImportError):
        pf.lib()


@pytest.mark.parametrize("prec,esz", [("fp32", 4), ("fp64", 8)])
def test_largest_addressable_grid(prec, esz):
    """A plane of the state must span < 4 GiB (32-bit per-lane offsets within a
    buffer group): a plane of one z row less passes the size check (and then
    fails without a device, PF_EHIP, or makes a handle where there is one), a
    4 GiB plane is PF_EUNSUPPORTED."""
    L = pf.lib()
    limit = (1 << 32) // esz  # cells of a 4 GiB plane
    nx = ny = 1024
    for nz, refused in ((limit // (nx * ny) - 1, False), (limit // (nx * ny), True)):
        d = dict(dim=3, nx=nx, ny=ny, nz=nz, n_phi=2, type_of=[0, 0], n_types=1, dx=1.0, W=3.0,
                 gamma=[1.0], mob=[1.0], k=[500.0], c0=[0.5], D=[1.0], with_c=True)
        keep = []
        p = pf._cparams(d, prec, 5, keep)
        h = C.c_void_p()
        rc = L.pf_create(C.byref(p), C.byref(h))
        if h.value:
            L.pf_destroy(h)
        if refused:
            assert rc == -7 and not h.value, (prec, nz, rc)
        else:
            assert rc in (0, -2), (prec, nz, rc)


def test_header_is_plain_c(tmp_path):
    """include/pf.h is a C header: a C99 program (-pedantic, warnings as errors)
    includes it, links libpf.so and calls it without a device."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = tmp_path / "c_abi.c"
    src.write_text('#include "pf.h"\n'
                   "int main(void) {\n"
                   "    pf_stats st;\n"
                   "    pf_controller c;\n"
                   "    double h = 0.0;\n"
                   "    int last = 0;\n"
                   "    (void)st;\n"
                   "    if (pf_create(0, 0) != PF_EINVAL) return 1;\n"
                   "    if (pf_controller_init(&c) != PF_OK) return 2;\n"
                   "    if (pf_clip_step(0.0, 1.0, 0.4, &h, &last) != 1 || h != 0.4 || last) return 3;\n"
                   "    return 0;\n"
                   "}\n")
    lib_dir = os.path.dirname(pf.LIB_PATH)
    exe = tmp_path / "c_abi"
    cmd = [gcc, "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
           str(src), "-L", lib_dir, "-l:libpf.so", f"-Wl,-rpath,{lib_dir}", "-o", str(exe)]
    p = subprocess.run(cmd, capture_output=True, text=True)
    assert p.returncode == 0, p.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stderr)
