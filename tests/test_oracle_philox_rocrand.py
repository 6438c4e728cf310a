"""The oracle's Philox4x32-10 against an independent implementation of the
published generator (Salmon et al., SC'11): AMD's rocRAND engine, built here
from its headers for the host and driven through its public interface.

rocRAND's engine with seed s, subsequence q and offset 4 o returns, in its
next four draws, the four words of Philox4x32-10 at key (s mod 2^32, s >> 32)
and counter (o mod 2^32, o >> 32, q mod 2^32, q >> 32).  No GPU is used.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

INCLUDE = "/opt/rocm/include"

PROGRAM = r'''
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>
int main() {
    unsigned long long s, q, o;
    while (std::scanf("%llu %llu %llu", &s, &q, &o) == 3) {
        rocrand_device::philox4x32_10_engine e(s, q, 4ull * o);
        const unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
'''


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None or not os.path.exists(os.path.join(INCLUDE, "rocrand",
                                                         "rocrand_philox4x32_10.h")):
        pytest.skip("rocRAND headers or hipcc not available")
    d = tmp_path_factory.mktemp("rocrand")
    src = d / "philox_kat.cpp"
    exe = d / "philox_kat"
    src.write_text(PROGRAM)
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-I", INCLUDE,
                        str(src), "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not build the rocRAND probe: " + r.stderr[-300:])

    def run(cases):
        inp = "".join(f"{s} {q} {o}\n" for s, q, o in cases)
        out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True,
                             check=True).stdout.split()
        return np.array(out, dtype=np.uint64).astype(np.uint32).reshape(-1, 4)
    return run


def _cases():
    g = np.random.default_rng(11)
    cases = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1),
             (0xFFFFFFFFFFFFFFFF, 0xFFFFFFFFFFFFFFFF, (1 << 30) - 1),
             (0x0123456789ABCDEF, 42 | (3 << 32), 77)]
    for _ in range(40):
        cases.append((int(g.integers(0, 2 ** 63)) * 2 + int(g.integers(0, 2)),
                      int(g.integers(0, 2 ** 63)) * 2 + int(g.integers(0, 2)),
                      int(g.integers(0, 2 ** 62))))
    return cases


def test_oracle_philox_equals_rocrand(orc, rocrand_philox):
    cases = _cases()
    ref = rocrand_philox(cases)
    for (s, q, o), want in zip(cases, ref):
        ctr = np.array([o & 0xFFFFFFFF, o >> 32, q & 0xFFFFFFFF, q >> 32], dtype=np.uint32)
        key = np.array([s & 0xFFFFFFFF, s >> 32], dtype=np.uint32)
        assert np.array_equal(orc.philox4x32(ctr, key), want), (s, q, o)


def test_noise_counter_layout_equals_rocrand(orc, rocrand_philox):
    """The oracle's draws for particle id at step t, replica r and purpose p
    are Philox at counter (id, t, r, p) and key = seed: rocRAND's subsequence
    r + p 2^32 and offset 4 (id + t 2^32)."""
    seed, step, replica, purpose = 0xDEADBEEF12345678, 9, 5, 1
    ids = np.arange(0, 5000, 97, dtype=np.uint32)
    got = orc.philox_batch(seed, ids, step=step, replica=replica, purpose=purpose)
    ref = rocrand_philox([(seed, replica | (purpose << 32), int(i) | (step << 32)) for i in ids])
    assert np.array_equal(got, ref)
