"""Host logic of bench.py (no GPU): the algorithmic byte counts behind the
roofline, the staleness rule of the stored HBM traffic, and the one-GPU
refusal."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_of_the_push():
    # binary64 3D: read cell 4 + offsets 24 + four-velocity 24 + m, q/mc 16,
    # write cell 4 + offsets 24 + four-velocity 24; per cell E, B 48 + the
    # accumulated -dM, -dE_k read and written 64 + n_CR, J_CR written 32
    a = bench.algorithmic_bytes(3, 4_194_304, 64 ** 3)
    assert a["per_particle"] == 120 and a["per_cell"] == 144
    assert a["per_launch"] == 541_065_216
    b = bench.algorithmic_bytes(2, 16_777_216, 8192 * 32)
    assert b["per_particle"] == 104
    assert b["per_launch"] == 1_782_579_200
    c = bench.algorithmic_bytes(3, 10, 0, fsz=4, msz=4)
    assert c["per_particle"] == (4 + 12 + 12 + 8) + (4 + 12 + 12)


def test_algorithmic_bytes_when_the_push_moves_the_particles():
    # the push also reads the slot map (4) and writes m and q/mc at the new
    # slot (2 * msz)
    a = bench.algorithmic_bytes(3, 4_194_304, 64 ** 3, moves_in_push=True)
    assert a["per_particle"] == 140 and a["per_cell"] == 144
    assert a["per_launch"] == 4_194_304 * 140 + 64 ** 3 * 144
    b = bench.algorithmic_bytes(2, 16_777_216, 8192 * 32, moves_in_push=True)
    assert b["per_particle"] == 124
    c = bench.algorithmic_bytes(3, 10, 0, fsz=4, msz=4, moves_in_push=True)
    assert c["per_particle"] == 76
    # the library moves the particles in the push unless told otherwise
    assert bench.moves_in_push(3, 0) and bench.moves_in_push(2, 0) and bench.moves_in_push(2, 2)
    assert not bench.moves_in_push(3, 1)


def test_stored_traffic_follows_the_kernel_sources(monkeypatch, tmp_path):
    label = "bell3d-64^3-ppc16-hall"
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps(
        {label: {"kernel_hash": bench.kernel_hash(), "bytes_per_launch": 123}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic(label, 1.0) == 123
    assert bench.load_traffic("no-such-workload", 1.0) is None
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0000000000000000")
    assert bench.load_traffic(label, 1.0) is None  # sources changed: no stale traffic


def test_kernel_hash_covers_every_source_file():
    h = bench.kernel_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert sorted(os.listdir(bench.CSRC))  # hashed in name order


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
