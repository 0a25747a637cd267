"""CPU model check of the one-barrier rounds of the shuffle.

tests/rounds1_model.cc restates the round protocol of rounds1_body (check and
commit round r, then refill by quota and reserve round r+1, one gather
barrier; hashed priority slots with round tags and a reset every tag cycle,
a dense window with three parities, the top active swap committing
regardless, records read early or late) with one host thread per workgroup
and no barrier between a round's checks and the next round's reservations.
Under random interleavings, and an adversarial schedule in which workgroup 0
checks a round only after every other workgroup reserved the next one, the
output must equal the sequential Knuth shuffle of §4.1 with the same targets.
Two planted mistakes must be caught: clearing the window parity still being
checked, and resetting the table without first waiting for every check of
the old tags.  CPU only: g++.
"""
import os
import random
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rounds1_model.cc")
RANKMAX = (1 << 24) - 1

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


@pytest.fixture(scope="module")
def model_src():
    with open(SRC) as f:
        return f.read()


def _build(tmp_path, name, text):
    src = str(tmp_path / (name + ".cc"))
    with open(src, "w") as f:
        f.write(text)
    exe = str(tmp_path / name)
    res = subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-o", exe, src],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    return exe


def _run(exe, seed, cfg):
    return subprocess.run([exe, str(seed), *map(str, cfg)], capture_output=True, text=True,
                          timeout=120)


# n, workgroups, lanes, k, table slots, chunk_log2, tag cycle, rank limit, early, adversarial
CONFIGS = [
    (3000, 4, 64, 96, 96, 0, 256, RANKMAX, 0, 0),
    (3000, 4, 64, 96, 96, 0, 256, RANKMAX, 1, 1),     # early records, slow checker
    (5000, 8, 64, 200, 100, 1, 4, 300, 0, 1),         # rank throttle, frequent resets
    (4000, 6, 32, 80, 40, 0, 2, RANKMAX, 1, 1),       # a reset every other round
    (6000, 12, 64, 384, 384, 2, 8, RANKMAX, 0, 1),    # chunks of 4
    (2000, 1, 128, 60, 60, 0, 16, RANKMAX, 0, 0),     # one workgroup
    (777, 3, 16, 20, 5, 0, 3, RANKMAX, 1, 0),         # a tiny table: most checks collide
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: "n%d_G%d_k%d" % (c[0], c[1], c[3]))
def test_rounds1_protocol(tmp_path, model_src, cfg):
    exe = _build(tmp_path, "model", model_src)
    for seed in (1, 2, 3):
        res = _run(exe, seed, cfg)
        assert res.returncode == 0 and res.stdout.startswith("ok:"), (seed, res.stdout,
                                                                      res.stderr)
        if cfg[7] != RANKMAX:
            assert " 0 throttled" not in res.stdout, res.stdout


def _random_shapes(count, seed=2103):
    """Shapes drawn over wide ranges, degenerate ones included: 1-12
    workgroups, tables of a quarter to twice k slots, tag cycles down to 2,
    rank limits down to the first refill's size."""
    rnd = random.Random(seed)
    out = []
    for _ in range(count):
        G = rnd.choice([1, 2, 3, 4, 6, 8, 12])
        L = rnd.choice([16, 32, 64, 128])
        k = rnd.randint(G, max(G, G * L // 2))
        T = max(1, int(k * rnd.choice([0.25, 0.5, 1.0, 2.0])))
        cl = rnd.choice([0, 0, 1, 2])
        tc = rnd.choice([2, 3, 8, 256])
        cap = rnd.choice([RANKMAX, RANKMAX, 2 * k + 5, k + 1, 50])
        n = rnd.randint(2, 6000)
        out.append((rnd.randint(1, 10**9),
                    (n, G, L, k, T, cl, tc, cap, rnd.randint(0, 1), rnd.randint(0, 1))))
    return out


def test_rounds1_protocol_random_shapes(tmp_path, model_src):
    """RP_MODEL_SHAPES (default 40) shapes from a fixed generator; a longer
    sweep is the same test with a larger count."""
    exe = _build(tmp_path, "model", model_src)
    for seed, cfg in _random_shapes(int(os.environ.get("RP_MODEL_SHAPES", "40"))):
        res = _run(exe, seed, cfg)
        assert res.returncode == 0 and res.stdout.startswith("ok:"), (seed, cfg, res.stdout,
                                                                      res.stderr)


MISTAKES = {
    # round r+1 clears the parity its slow peers still check for round r
    "window_parity": ("const uint32_t cp = (uint32_t)((rr + 1) % PAR);",
                      "const uint32_t cp = (uint32_t)((rr + 2) % PAR);",
                      (3000, 4, 64, 96, 96, 0, 256, RANKMAX, 0, 1)),
    # the table reset without the barrier that waits for the old tags' checks
    "reset_barrier": ("""            if (!barrier(w, ++epoch, Pay{}, nullptr, nullptr))
                return;
            for (uint32_t i = w; i < C.T; i += G)""",
                      """            for (uint32_t i = w; i < C.T; i += G)""",
                      (3000, 4, 64, 96, 96, 0, 2, RANKMAX, 0, 0)),
}


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_model_catches_a_planted_mistake(tmp_path, model_src, name):
    right, wrong, cfg = MISTAKES[name]
    assert model_src.count(right) == 1
    exe = _build(tmp_path, "variant", model_src.replace(right, wrong))
    outs = []
    for seed in range(1, 6):
        res = _run(exe, seed, cfg)
        outs.append(res.stdout.strip())
        if res.returncode == 1 and "violation" in res.stdout:
            return
    pytest.fail("planted mistake %s not caught: %s" % (name, outs))
