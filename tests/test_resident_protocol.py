"""CPU model check of the resident serving kernel's claim and gang protocol.

tests/resident_model.cc restates the protocol of rp_resident_kernel (claim in
ring order, gangs formed from idle workgroups under a locked gang word, the
last member to see a gang full clears it, a leader hands back a gang that has
not formed in time) with host threads and std::atomic, and checks under random
interleavings that every request runs exactly once, every gang has exactly its
members, a handed-back request never ran, and everything ends.  A second run
plants a mistake in the model (the first member to see its gang full clears
the word, not the last) and must be caught.  CPU only: g++.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "resident_model.cc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def _build(tmp_path, source_text=None):
    src = SRC
    if source_text is not None:
        src = str(tmp_path / "model_variant.cc")
        with open(src, "w") as f:
            f.write(source_text)
    exe = str(tmp_path / ("model_variant" if source_text is not None else "model"))
    res = subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-o", exe, src],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    return exe


# seed, workers, requests, ring entries, largest gang, gang formation limit (us)
CONFIGS = [
    (1, 16, 400, 64, 8, 2000),     # gangs form in time
    (2, 8, 300, 16, 8, 200),       # a small ring that wraps often, gangs of the whole grid
    (3, 32, 600, 64, 16, 1000),
    (4, 16, 300, 8, 16, 0),        # no time to form: every gang is handed back
    (5, 4, 200, 16, 4, 50),
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: "seed%d" % c[0])
def test_protocol_model(tmp_path, cfg):
    exe = _build(tmp_path)
    res = subprocess.run([exe, *map(str, cfg)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok:"), res.stdout
    if cfg[5] == 0:
        # every gang was handed back and ran on one workgroup instead
        assert " 0 gangs handed back" not in res.stdout


def test_model_catches_a_planted_mistake(tmp_path):
    text = open(SRC).read()
    right = """            if (c.gang_left.fetch_add(1) + 1 == need) {"""
    assert text.count(right) == 1
    exe = _build(tmp_path, text.replace(right, """            if (c.gang_left.fetch_add(1) == 0) {"""))
    res = subprocess.run([exe, "1", "16", "400", "64", "8", "2000"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 1 and "violation" in res.stdout, res.stdout
