"""The oracle's Philox4x32-10 (written from Salmon et al., SC'11) against
rocRAND's implementation of the same generator, on random counters and
keys: a library routine, independent of both the oracle and the GPU
library.  CPU only (the helper is host code built with hipcc)."""
import os
import random
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists(HEADER):
        pytest.skip("hipcc or the rocRAND headers are not installed")
    exe = str(tmp_path_factory.mktemp("rocrand") / "philox_ref")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-o", exe,
                    os.path.join(HERE, "rocrand_philox_ref.cpp")], check=True,
                   capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_ref):
    g = random.Random(1701)
    cases = [[g.getrandbits(32) for _ in range(6)] for _ in range(2000)]
    cases += [[0] * 6, [0xFFFFFFFF] * 6, [1, 0, 0, 0, 0, 0], [0, 0, 0, 0, 1, 0]]
    text = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True, check=True)
    got = [list(map(int, line.split())) for line in out.stdout.strip().splitlines()]
    assert len(got) == len(cases)
    for c, want in zip(cases, got):
        assert orc.philox4x32_10(c[:4], c[4:]) == want, c
