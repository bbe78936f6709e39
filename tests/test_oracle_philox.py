"""Pin for the oracle's Philox4x32-10 (Salmon et al., SC'11) against a library
routine: rocRAND's block function, compiled here from its open-source header."""
import hashlib
import os
import random
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

HELPER = os.path.join(os.path.dirname(__file__), "helpers", "philox_rocrand.cpp")


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to compile the rocRAND reference")
    tag = hashlib.sha1(open(HELPER, "rb").read()).hexdigest()[:12]
    exe = os.path.join(tempfile.gettempdir(), f"philox_rocrand_{tag}")
    if not os.path.exists(exe):
        subprocess.check_call([hipcc, "-O1", "--offload-arch=gfx950", "-o", exe + ".tmp", HELPER],
                              cwd=tempfile.gettempdir())
        os.replace(exe + ".tmp", exe)

    def run(rows):
        text = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return [list(map(int, line.split())) for line in out.strip().splitlines()]
    return run


def test_against_rocrand(orc, rocrand_ref):
    rng = random.Random(11)
    rows = [[0] * 6, [2**32 - 1] * 6]
    rows += [[rng.randrange(2**32) for _ in range(6)] for _ in range(500)]
    rows += [[s, a, it, 0, 7, 0] for s in range(4) for a in range(3) for it in range(3)]
    ref = rocrand_ref(rows)
    for r, want in zip(rows, ref):
        got = orc.philox4x32_10(r[:4], r[4:])
        assert list(map(int, got)) == want, r


def test_draw_mapping(orc):
    # word 0 of the block at counter (step, ant, iteration, 0), key (seed lo, seed hi)
    seed = 0x1234_5678_9ABC_DEF0
    for (it, ant, step) in [(0, 0, 0), (3, 17, 999), (49, 255, 19_999)]:
        w = orc.philox4x32_10([step, ant, it, 0], [seed & 0xFFFFFFFF, seed >> 32])[0]
        assert orc.draw(seed, it, ant, step) == int(w)
        w0 = orc.philox4x32_10([0, ant, it, 0], [seed & 0xFFFFFFFF, seed >> 32])[0]
        n = 20_000
        assert orc.start_city(seed, it, ant, n) == (int(w0) * n) >> 32   # start uses step 0


def test_start_city_uniformity(orc):
    # multiply-shift start is uniform up to 2^-32; check histogram over many ants
    n = 7
    counts = np.bincount([orc.start_city(5, 0, a, n) for a in range(14_000)], minlength=n)
    exp = 14_000 / n
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 30.0   # 6 dof; p ~ 4e-5
