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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_solve_descriptor_validation():
    """Empty and out-of-range descriptors are refused before any device work
    (workspace size 0 and the reason in fcgno_last_error)."""
    import paper_2402_05598_amd._binding as b
    ok = dict(n=32, batch=2, op="identity", m_max=5, max_iter=100, rtol=1e-6)
    assert b.solve_workspace_bytes(None, **{**ok, "n": 32}) > 0
    bad = [dict(n=0), dict(batch=0), dict(m_max=0), dict(m_max=33), dict(max_iter=0), dict(rtol=0.0),
           dict(rtol=-1.0), dict(rtol=float("nan")), dict(op="bf16"), dict(op="fp64")]
    for d in bad:
        assert b.solve_workspace_bytes(None, **{**ok, **d}) == 0, d
    # the iteration history and window storage grow with max_iter and m_max
    a = b.solve_workspace_bytes(None, **ok)
    assert b.solve_workspace_bytes(None, **{**ok, "max_iter": 1000}) > a
    assert b.solve_workspace_bytes(None, **{**ok, "m_max": 20}) > a
    lib = b.lib()
    d = b.SolveDesc(32, 2, 5, 100, 1e-6, 99, 0, 1)
    assert lib.fcgno_solve_workspace_bytes(None, ctypes.byref(d)) == 0
    assert b"unknown op" in lib.fcgno_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_streams_field_range():
    import paper_2402_05598_amd._binding as b
    lib = b.lib()
    for streams, ok in ((0, True), (1, True), (8, True), (9, False), (-1, False)):
        d = b.SolveDesc(32, 4, 5, 100, 1e-6, b.OP["identity"], 0, 1, streams)
        assert (lib.fcgno_solve_workspace_bytes(None, ctypes.byref(d)) > 0) == ok, streams


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_status_strings_and_engine_footprint():
    """Host-only entry points: every status has a name; the serving engine's
    per-request footprint (the basis of admission) grows with the grid, the
    iteration limit and the window, and is refused for invalid requests."""
    import paper_2402_05598_amd._binding as b
    lib = b.lib()
    lib.fcgno_status_string.argtypes = [ctypes.c_int]
    lib.fcgno_status_string.restype = ctypes.c_char_p
    names = {s: lib.fcgno_status_string(s) for s in (0, 1, -1, -2, -3)}
    assert all(names.values()) and len(set(names.values())) == 5
    d = b.EngineDesc(b.OP["identity"], 5, 8, 16, 1 << 30)
    f = lambda n, it: lib.fcgno_engine_request_bytes(None, ctypes.byref(d), n, it)
    assert 0 < f(64, 300) < f(128, 300) < f(256, 300)
    assert f(128, 300) < f(128, 3000)
    d20 = b.EngineDesc(b.OP["identity"], 20, 8, 16, 1 << 30)
    assert lib.fcgno_engine_request_bytes(None, ctypes.byref(d20), 128, 300) > f(128, 300)
    assert f(0, 300) == 0 and f(64, 0) == 0
    # a neural-operator request needs a model
    dn = b.EngineDesc(b.OP["bf16"], 5, 8, 16, 1 << 30)
    assert lib.fcgno_engine_request_bytes(None, ctypes.byref(dn), 64, 300) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_size_limits_at_every_entry_point():
    """Grids above 32768 per side or batches above 65535 are refused before any
    device work: workspace queries give 0 and calls give FCGNO_E_INVALID with
    the reason (the kernels index a system with 32-bit products and launch
    one grid row per system)."""
    import paper_2402_05598_amd._binding as b
    lib = b.lib()
    lib.fcgno_krylov_samples_workspace_bytes.restype = ctypes.c_size_t
    lib.fcgno_energy_loss_workspace_bytes.restype = ctypes.c_size_t
    lib.fcgno_krylov_samples.restype = ctypes.c_int
    ok = dict(n=64, batch=2, op="identity", m_max=5, max_iter=100, rtol=1e-6)
    assert b.solve_workspace_bytes(None, **ok) > 0
    assert b.solve_workspace_bytes(None, **{**ok, "n": 32768, "batch": 1}) > 0
    for d in (dict(n=32769, batch=1), dict(n=8, batch=65536)):
        assert b.solve_workspace_bytes(None, **{**ok, **d}) == 0, d
    assert lib.fcgno_krylov_samples_workspace_bytes(64, 2, 10) > 0
    assert lib.fcgno_krylov_samples_workspace_bytes(32769, 1, 10) == 0
    assert lib.fcgno_krylov_samples_workspace_bytes(8, 65536, 10) == 0
    assert lib.fcgno_energy_loss_workspace_bytes(64, 2) > 0
    assert lib.fcgno_energy_loss_workspace_bytes(32769, 1) == 0
    assert lib.fcgno_energy_loss_workspace_bytes(8, 65536) == 0
    # a call with sizes out of range fails on the host, before its pointers are used
    vp = ctypes.c_void_p(1)
    st = lib.fcgno_krylov_samples(ctypes.c_int32(32769), ctypes.c_int32(1), ctypes.c_int32(4), ctypes.c_int32(10),
                                  vp, vp, vp, vp, vp, vp, ctypes.c_size_t(1 << 40), None)
    assert st == -1 and b"32768" in lib.fcgno_last_error()
    d = b.EngineDesc(b.OP["identity"], 5, 8, 16, 1 << 30)
    f = lambda n: lib.fcgno_engine_request_bytes(None, ctypes.byref(d), n, 300)
    assert f(64) > 0 and f(32769) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_model_and_training_arguments_refused_on_the_host():
    """Unsupported architectures, wrong weight counts, non-finite weights,
    unknown losses and training precisions are refused before any device
    call, each with its reason."""
    import numpy as np
    import paper_2402_05598_amd._binding as b
    lib = b.lib()

    def create(layers=4, width=32, modes=12, cin=4, basis=0, count=None, bad=None):
        a = b.Arch(layers, width, modes, cin, basis)
        n = int(lib.fcgno_weight_count(ctypes.byref(a))) if count is None else count
        w = np.zeros(max(n, 1))
        if bad is not None:
            w[bad] = np.nan
        h = ctypes.c_void_p()
        st = lib.fcgno_model_create(ctypes.byref(a), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n,
                                    ctypes.byref(h))
        return st, lib.fcgno_last_error()

    # the blob size follows the layout in the header
    a = b.Arch(4, 32, 12, 4, 0)
    C, M, L = 32, 12, 4
    assert lib.fcgno_weight_count(ctypes.byref(a)) == C * 4 + C + L * (2 * C * C * 2 * M * M + C * C + C) + C + 1
    for kw, why in ((dict(width=24), b"width"), (dict(modes=17), b"modes"), (dict(modes=0), b"modes"),
                    (dict(cin=3), b"in_channels"), (dict(basis=2), b"basis"), (dict(layers=0), b"layers"),
                    (dict(count=10), b"weight count"), (dict(bad=5), b"non-finite")):
        st, msg = create(**kw)
        assert st == -1 and why in msg, (kw, msg)
    # losses and training precisions
    lib.fcgno_loss.restype = ctypes.c_int
    vp = ctypes.c_void_p(1)
    st = lib.fcgno_loss(ctypes.c_int32(7), ctypes.c_int32(8), ctypes.c_int32(1), vp, vp, vp, vp, None, vp,
                        ctypes.c_size_t(1 << 30), None)
    assert st == -1 and b"unknown loss" in lib.fcgno_last_error()
    lib.fcgno_train_workspace_bytes.restype = ctypes.c_size_t
    assert lib.fcgno_train_workspace_bytes(None, 32, 2, 1) == 0
    assert b"null model" in lib.fcgno_last_error()


def test_kernel_parameters_use_generic_pointers():
    """The host pass sees the global-address-space qualifier as empty, so a
    kernel parameter carrying it would make the host register the kernel under
    a name (mangled without the qualifier) that the device code object does
    not hold, and its first launch would fail.  Qualified pointers belong in
    kernel bodies and structs, not in kernel parameter lists."""
    csrc = os.path.join(ROOT, "paper_2402_05598_amd", "csrc")
    bad = []
    for fn in sorted(os.listdir(csrc)):
        if not fn.endswith(".hip"):
            continue
        text = open(os.path.join(csrc, fn)).read()
        for m in re.finditer(r"__global__[^{;]*?\bk_\w+\s*\(([^)]*)\)", text, flags=re.S):
            if re.search(r"\bGLOBAL\b", m.group(1)):
                bad.append((fn, m.group(0)[:80]))
    assert not bad, bad
