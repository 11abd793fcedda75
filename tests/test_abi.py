"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every function
that include/nbody.h declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_2604_09184_amd as nb
    if not os.path.exists(nb.LIB_PATH):
        pytest.fail("libnbody.so not built")
    return nb.lib()


def test_header_declares_the_boundary():
    names = declared()
    for req in ("nbody_kick", "nbody_drift", "nbody_encounters", "nbody_step", "nbody_rcrit",
                "nbody_jump", "nbody_create", "nbody_destroy"):
        assert req in names


def test_every_declared_symbol_is_exported(L):
    import paper_2604_09184_amd as nb
    out = subprocess.run(["nm", "-D", "--defined-only", nb.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (nbody_[a-z_]+)\b", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        assert hasattr(L, n)


def test_binding_covers_the_boundary():
    import paper_2604_09184_amd as nb
    covered = set(nb.EXPORTS) | set(nb.OTHER_EXPORTS)
    assert set(declared()) <= covered


def test_invalid_arguments_rejected_on_host(L):
    import paper_2604_09184_amd as nb
    h = ctypes.c_void_p()
    assert L.nbody_create(ctypes.byref(h), ctypes.byref(nb.Params().c())) == 0
    try:
        E_INVAL = -1
        # n <= 0
        assert L.nbody_kick(h, 0, None, None, None, 0.0, None, None, None) == E_INVAL
        assert L.nbody_drift(h, -5, None, None, 0.0, None, None) == E_INVAL
        # required pointers
        assert L.nbody_kick(h, 10, None, None, None, 0.0, None, None, None) == E_INVAL
        assert b"xm" in L.nbody_last_error(h)
        assert L.nbody_encounters(h, 10, None, None, None, 0, None, None) == E_INVAL
        assert L.nbody_step(h, 10, None, None, None, 1, None, 0, None, None, None) == E_INVAL
        assert L.nbody_validate(h, 10, None, None, None, None) == E_INVAL
        assert L.nbody_reserve(h, 10, 8, None) == E_INVAL          # unknown reservation flag
        assert b"flags" in L.nbody_last_error(h)
        assert L.nbody_reserve(h, 0, 1, None) == E_INVAL
        assert L.nbody_validate(h, 0, 64, 64, 64, None) == E_INVAL
        # misaligned pointer is refused before any device call
        assert L.nbody_rcrit(h, 10, 8, 8, 8, None) == E_INVAL
        assert b"aligned" in L.nbody_last_error(h)
        # bad parameters
        bad = nb.Params(m0=-1.0).c()
        assert L.nbody_set_params(h, ctypes.byref(bad)) == E_INVAL
        bad = nb.Params(f_in=1.5).c()
        assert L.nbody_set_params(h, ctypes.byref(bad)) == E_INVAL
    finally:
        assert L.nbody_destroy(h) == 0
    assert L.nbody_create(None, None) == -1


def test_version_string(L):
    assert b"gfx950" in L.nbody_version()


def test_library_does_not_link_the_oracle():
    import paper_2604_09184_amd as nb
    out = subprocess.run(["ldd", nb.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in out
    src_dir = os.path.join(ROOT, "paper_2604_09184_amd")
    for dirpath, _, files in os.walk(src_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text, f


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    """No CPU fallback: with the shared library absent the binding raises."""
    import paper_2604_09184_amd as nb
    monkeypatch.setattr(nb, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(nb, "_lib", None)
    with pytest.raises(nb.NBodyError):
        nb.lib()
    with pytest.raises(nb.NBodyError):
        nb.Context(nb.Params())
