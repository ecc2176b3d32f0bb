"""Host-side parts of bench.py (no GPU): the algorithmic byte count behind
the roofline figure, the kernel-source hash that invalidates stale traffic
counters, and the refusal of more than one GPU."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_inner_layer_algorithmic_bytes():
    """BF16 inner layer at C = 32, M = 12 (MP = 32), N = 512, one segment per
    row: read and write [point][C] in 2-byte elements (128 B/pt) plus per row
    the synthesis operand [C][MP] (2 B) and the partial spectra of the 2M = 24
    kept mode slots [24][C] (4 B): 138 bytes per point, 36 175 872 bytes per
    system."""
    b = _bench()
    per_sys = b.layer_bytes_per_launch(512, 1, 32, 12, 2, 4, 1)
    assert per_sys == 512 * (512 * 128 + 32 * 32 * 2 + 24 * 32 * 4) == 36175872
    assert per_sys / 512 ** 2 == 138.0
    # linear in the batch; M = 4 rounds MP up to 16 (FP32 stores all MP slots);
    # two segments double the partials
    assert b.layer_bytes_per_launch(512, 16, 32, 12, 2, 4, 1) == 16 * per_sys
    assert b.layer_bytes_per_launch(64, 1, 16, 4, 4, 4, 1) == 64 * (64 * 2 * 16 * 4 + 16 * 16 * 4 + 16 * 16 * 4)
    two_seg = b.layer_bytes_per_launch(1024, 1, 32, 12, 2, 4, 2)
    assert two_seg - 1024 * (1024 * 128 + 2048) == 1024 * 2 * 24 * 32 * 4


def test_kernel_hash_tracks_the_layer_sources():
    b = _bench()
    h = b.kernel_hash()
    assert len(h) == 16 and h == b.kernel_hash()
    assert all(os.path.exists(os.path.join(ROOT, rel)) for rel in b.KERNEL_SOURCES)


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode != 0
    assert "one GPU" in (out.stdout + out.stderr)
