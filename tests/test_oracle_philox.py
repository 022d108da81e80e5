"""Pins for the oracle's Philox4x32-10 (the random stream both sides follow).

* published known-answer vectors (tests/golden/philox4x32_10_kat.txt);
* a second implementation on Python integers (oracle/pure.py);
* rocRAND's Philox4x32-10 engine, compiled from its header for the host CPU,
  with the counter/key mapping of its (seed, subsequence, offset) constructor.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import pure

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(s, 16) for s in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_kat_c(oracle_mod):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle_mod.philox(ctr, key) == out


def test_kat_python():
    for ctr, key, out in _kat_rows():
        assert pure.philox4x32_10(ctr, key) == out


def test_c_vs_python_random(oracle_mod):
    rng = np.random.default_rng(11)
    for _ in range(2000):
        ctr = [int(v) for v in rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)]
        assert oracle_mod.philox(ctr, key) == pure.philox4x32_10(ctr, key)


_ROCRAND_PROG = r"""
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
    unsigned long long offset = 4ull * (((unsigned long long)c1 << 32) | c0);
    rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
    uint4 r = e.next4();
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_c_vs_rocrand_host(oracle_mod, tmp_path):
    src = tmp_path / "kat.hip"
    src.write_text(_ROCRAND_PROG)
    exe = tmp_path / "kat"
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-O1", "-o", str(exe), str(src)], check=True,
                   capture_output=True)
    rng = np.random.default_rng(5)
    cases = [[int(v) for v in rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)] for _ in range(300)]
    # rocRAND's offset is 4 * (ctr1:ctr0) in 64 bits: keep ctr1 below 2^30 so it does not wrap
    for c in cases:
        c[1] &= (1 << 30) - 1
    inp = "\n".join(" ".join(f"{v:08x}" for v in c) for c in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        got = [int(s, 16) for s in line.split()]
        assert got == oracle_mod.philox(c[0:4], c[4:6])
