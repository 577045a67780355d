"""Host-side code under the address and undefined-behaviour sanitizers (no GPU).

* The library's host checks (``csrc/checks.h``: size limits and the pass
  watchdog bound) are built with g++ into a small driver
  (``tests/native/host_checks.cpp``).  The watchdog bound must equal the
  exact least K with (num+den)^K >= n den^K (Section 3.1: each pass that
  leaves survivors shrinks |V| by more than the factor 1 + eps), capped at n,
  computed here with Python integers (where the powers stay below a few
  million bits; beyond that, equal to the rounded-up floating-point
  quotient ln n / ln(1+eps), which is then far from an integer).
* The C oracles are built with gcc and run by ``tests/native/oracle_driver.c``
  over generated graphs and inputs that break the CSR contract.
* A CSR whose rows are one-sided drives the oracle, through its Python
  wrapper, to its internal-error status.
"""
from __future__ import annotations

import math
import os
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

import oracle

ROOT = Path(__file__).resolve().parents[1]
NATIVE = ROOT / "tests" / "native"
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _compile(tmp_path, compiler, sources, out, extra=()):
    exe = tmp_path / out
    cmd = [compiler, *SAN, *extra, *map(str, sources), "-o", str(exe)]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    assert proc.returncode == 0, proc.stdout + proc.stderr
    return exe


def _run(exe, stdin=None, args=()):
    env = dict(os.environ, UBSAN_OPTIONS="print_stacktrace=1")
    proc = subprocess.run([str(exe), *args], input=stdin, capture_output=True, text=True,
                          env=env, timeout=120)
    assert proc.returncode == 0, proc.stdout[-2000:] + proc.stderr[-4000:]
    return proc.stdout


def _exact_bound(n, num, den, max_bits=4_000_000):
    """Least K >= 1 with (num+den)^K >= n den^K, capped at n, or None when
    the powers would exceed max_bits bits.  A float estimate is moved to the
    least K that satisfies the exact integer condition."""
    if n <= 1:
        return max(n, 0)
    if num == 0:
        return n
    g = math.gcd(num, den)
    p, q = (num + den) // g, den // g

    def ok(k):
        return p ** k >= n * q ** k

    t = math.log(n) / math.log1p(num / den)
    if t > n * (1 + 1e-9) + 1:
        return n  # clearly (num+den)^(n-1) < n den^(n-1)
    k = max(1, math.ceil(t))
    if (min(k, n) + 1) * p.bit_length() > max_bits:
        return None
    while k < n and not ok(k):
        k += 1
    while k > 1 and ok(k - 1):
        k -= 1
    return min(n, k)


NS = [0, 1, 2, 3, 5, 10, 97, 1000, 10_000, 65_536, 100_000, 1_048_576, 2_000_000, 16_777_216,
      2_147_483_646]
EPS = [(0, 1), (1, 1000), (1, 100), (1, 20), (1, 10), (1, 3), (1, 2), (2, 3), (6, 4), (1, 1),
       (3, 1), (7, 2), (1000, 1), (2**40, 1), (2**62, 1), (1, 2**20)]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_pass_bound_and_size_checks_under_sanitizers(tmp_path):
    exe = _compile(tmp_path, "g++", [NATIVE / "host_checks.cpp"], "host_checks",
                   ["-std=c++17", f"-I{ROOT / 'paper_2103_00154_amd' / 'csrc'}",
                    f"-I{ROOT / 'include'}"])
    queries = [(n, num, den) for n in NS for (num, den) in EPS]
    size_cases = [  # (n, m, num, den) -> status
        ((10, 10, 1, 10), 0), ((0, 0, 0, 1), 0), ((-1, 0, 0, 1), -1), ((5, -1, 0, 1), -1),
        ((5, 5, -1, 1), -1), ((5, 5, 1, 0), -1), ((2**31 - 2, 0, 0, 1), 0),
        ((2**31 - 1, 0, 0, 1), -2), ((10, 2**30 - 1, 0, 1), 0), ((10, 2**30, 0, 1), -2),
        ((10, 1000, 2**62, 2**62), -2), ((10, 1, 2**62 - 2, 1), 0), ((10, 1, 2**62 - 1, 1), -2),
        ((2**31 - 2, 10, 1, 2**32), 0), ((2**31 - 2, 10, 1, 2**33), -2), ((1000, 10, 1, 2**40), 0)]
    text = "".join(f"b {n} {a} {b}\n" for n, a, b in queries)
    text += "".join(f"s {n} {m} {a} {b}\n" for (n, m, a, b), _ in size_cases)
    out = _run(exe, stdin=text).split("\n")
    fallback = 0
    for (n, num, den), line in zip(queries, out):
        tag, k, exact = line.split()
        k, exact = int(k), exact == "1"
        want = _exact_bound(n, num, den)
        if exact and want is None:  # powers too large here: the estimate's K
            t = math.log(n) / math.log1p(num / den)
            assert abs(t - round(t)) > 1e-6 and k == min(n, math.ceil(t)), (n, num, den, k)
        elif exact:
            assert k == want, (n, num, den, k, want)
        else:
            fallback += 1
            est = math.ceil(math.log(n) / math.log1p(num / den))
            if want is None:  # too long for the exact search here too
                assert min(n, est) <= k <= min(n, est + 2), (n, num, den, k)
            else:
                assert want <= k <= want + 2, (n, num, den, k, want)
    # the estimate decides (or the exact tie check settles) every case here
    assert fallback == 0, fallback
    for ((case, status), line) in zip(size_cases, out[len(queries):]):
        assert line == f"s {status}", (case, line)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracles_under_sanitizers(tmp_path):
    exe = _compile(tmp_path, "gcc",
                   [NATIVE / "oracle_driver.c", ROOT / "oracle" / "peel_oracle.c",
                    ROOT / "oracle" / "cbds_oracle.c"], "oracle_driver", ["-std=c11"])
    out = _run(exe, args=["1500"])
    assert out.startswith("ok 1500 graphs"), out


def test_one_sided_rows_are_an_oracle_internal_error():
    # vertices 1..10 list vertex 0, which lists only 1 and 2 (degree 2): pass
    # 1 removes 1..10 and decrements vertex 0 ten times, so |E| drops below 0
    rp = np.array([0, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12], np.int32)
    ci = np.array([1, 2] + [0] * 10, np.int32)
    assert oracle.check_csr(rp, ci, 11) < 0
    with pytest.raises(oracle.OracleError) as exc:
        oracle.peel(rp, ci, 11, 1, 10)
    assert exc.value.code == -3
    # a row listing a neighbour whose own row is empty: the last pass ends
    # with no vertex left but one edge counted
    rp = np.array([0, 2, 2, 2], np.int32)
    ci = np.array([1, 2], np.int32)
    with pytest.raises(oracle.OracleError) as exc:
        oracle.peel(rp, ci, 3, 0, 1)
    assert exc.value.code == -3
