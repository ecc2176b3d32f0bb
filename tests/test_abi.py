"""The C ABI library loads and exports every function include/fcgno.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcgno.h")
LIB = os.path.join(ROOT, "paper_2402_05598_amd", "libfcgno.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fcgno_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fcgno_solve", "fcgno_precond_apply", "fcgno_train_step", "fcgno_op_forward",
                     "fcgno_op_backward", "fcgno_energy_loss", "fcgno_model_create"):
        assert required in names, required


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (fcgno_[a-z_0-9]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2402_05598_amd._binding as b
    monkeypatch.setattr(b, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(b, "_lib", None)
    with pytest.raises(b.FcgnoError):
        b.lib()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_classical_preconditioner_descriptors():
    """JACOBI and SGS_RB take no model and need 1..1000 sweeps (host-side checks only)."""
    import paper_2402_05598_amd._binding as b
    assert b.solve_workspace_bytes(None, 32, 2, op="jacobi", precond_steps=4) > 0
    assert b.solve_workspace_bytes(None, 33, 1, op="sgs_rb", precond_steps=1) > 0
    for op in ("jacobi", "sgs_rb"):
        assert b.solve_workspace_bytes(None, 32, 2, op=op, precond_steps=0) == 0
        assert b.solve_workspace_bytes(None, 32, 2, op=op, precond_steps=1001) == 0
    # the Jacobi ping-pong iterate costs one more grid per system than SGS
    extra = (b.solve_workspace_bytes(None, 32, 2, op="jacobi", precond_steps=4)
             - b.solve_workspace_bytes(None, 32, 2, op="sgs_rb", precond_steps=4))
    assert extra >= 2 * 32 * 32 * 8
