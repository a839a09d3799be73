"""The scalar rules of the factorization kernels (csrc/rules.h: the
truncation rule of Sec. 2.3 with its discarded and kept weights, the Jacobi
convergence report) built for the host with the address and
undefined-behaviour sanitizers, run on spectra drawn here and compared with
the oracle's rank rule (oracle/mps.py truncation_rank, tail_sums).  CPU only."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import mps as om


@pytest.fixture(scope="module")
def rules_exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    from tests.host import sanitized_build
    return sanitized_build.build_rules_check(str(tmp_path_factory.mktemp("rules") / "rules_check"))


def run_cases(exe, lines):
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert r.returncode == 0, r.stderr
    return r.stdout.split("\n")[:len(lines)]


def t_line(s, mode, tol, max_rank, length, total=None):
    vals = " ".join(repr(float(x)) for x in s)
    return f"T {mode} {float(tol)!r} {max_rank} {length} {1 if total is not None else 0} " \
           f"{float(total) if total is not None else 0.0!r} {len(s)} {vals}"


def spectra(rng):
    out = []
    for _ in range(300):
        n = int(rng.integers(1, 200))
        kind = rng.integers(0, 5)
        if kind == 0:
            s = np.sort(np.abs(rng.standard_normal(n)))[::-1]
        elif kind == 1:
            s = np.exp(-np.arange(n) / rng.uniform(0.5, 30.0))
        elif kind == 2:
            s = np.exp(-np.arange(n) / rng.uniform(1.0, 10.0)) * rng.uniform(1e-3, 1e3)
            s[int(rng.integers(0, n)):] = 0.0  # exact zeros
        elif kind == 3:
            s = np.repeat(rng.uniform(0.1, 1.0), n)  # all equal
        else:
            s = np.sort(rng.uniform(0, 1, n) ** 8)[::-1]
        out.append(np.ascontiguousarray(s))
    return out


def test_truncation_rule_matches_the_oracle(rules_exe):
    rng = np.random.default_rng(2601)
    cases, lines = [], []
    for s in spectra(rng):
        for mode in (om.REL_NORM2, om.REL_SV):
            for tol in (0.0, 1e-14, 1e-12, 1e-10, 1e-6, 1e-2, 0.5):
                max_rank = int(rng.integers(1, len(s) + 3))
                cases.append((s, mode, tol, max_rank))
                lines.append(t_line(s, mode, tol, max_rank, len(s) + int(rng.integers(0, 3))))
    out = run_cases(rules_exe, lines)
    for (s, mode, tol, max_rank), o in zip(cases, out):
        tag, r, delta, kept = o.split()
        r = int(r)
        assert r == om.truncation_rank(s, tol, max_rank, mode), (len(s), mode, tol, max_rank)
        t = om.tail_sums(s)
        # same summation order as the oracle's tail: identical bits
        assert float(delta) == t[r]
        assert abs(float(kept) - float(np.sum(s[:r] ** 2))) <= 1e-15 * max(t[0], 1e-300) * len(s)


def test_truncation_rule_at_the_threshold_and_with_missed_weight(rules_exe):
    # tails placed exactly at tol * total: the rule keeps r with tail <= threshold
    s = np.array([1.0, 0.5, 0.25, 0.125, 0.0625])
    t = om.tail_sums(s)
    lines = [t_line(s, om.REL_NORM2, t[k] / t[0], 10, 5) for k in range(1, 5)]
    # an exact total larger than the values' own: the missed weight enters every tail
    lines.append(t_line(s, om.REL_NORM2, 0.0, 10, 5, total=t[0] + 0.01))
    lines.append(t_line(s, om.REL_NORM2, 0.02 / (t[0] + 0.01), 10, 5, total=t[0] + 0.01))
    out = run_cases(rules_exe, lines)
    for k, o in zip(range(1, 5), out[:4]):
        r = int(o.split()[1])
        assert r == om.truncation_rank(s, t[k] / t[0], 10)
        assert r <= k
    # missed 0.01 > tol * total = 0: nothing can be dropped, everything is kept
    _, r, delta, _ = out[4].split()
    assert int(r) == 5 and float(delta) == pytest.approx(0.01, rel=1e-12)
    # budget 0.02 on top of the 0.01 missed: only 0.0625^2 = 0.0039 fits
    _, r, delta, _ = out[5].split()
    assert int(r) == 4 and float(delta) == pytest.approx(0.01 + 0.0625 ** 2, rel=1e-12)


def test_jacobi_convergence_report(rules_exe):
    out = run_cases(rules_exe, ["J 0 40", "J 39 40", "J 40 40", "J 41 40", "J 3 3"])
    assert [o.split()[1] for o in out] == ["0", "0", "1", "1", "1"]
