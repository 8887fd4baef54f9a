"""The device math of the HIP evaluators (own sin/cos, exp/expm1 pair, Fermi and
Bose leaves with their mirrors and derivatives), compiled for the host with a
stand-in HIP header and compared with 40-digit mpmath values; the device
Philox generator and its momentum mapping against the oracle's and the
published known answers (CPU only)."""
import os
import shutil
import subprocess

import mpmath as mp
import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_math", "math_check.cpp")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("math") / "math_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-ffp-contract=off", "-I",
                    os.path.join(HERE, "cpu_math", "shim"), SRC, "-o", out], check=True)
    return out


def _run(exe, what, xs):
    res = subprocess.run([exe, what], input="\n".join(repr(float(x)) for x in xs),
                         capture_output=True, text=True, check=True)
    return np.array([[float(v) for v in line.split()] for line in res.stdout.splitlines()])


def _ulp_err(got, want):
    want = float(want)
    if want == 0.0:
        return abs(got)
    return abs(got - want) / abs(want) / 2.0 ** -52


def test_sincos_reduced(exe):
    mp.mp.dps = 40
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(-4 * np.pi, 4 * np.pi, 400), rng.uniform(-1e4, 1e4, 200),
                         [0.0, np.pi / 4, np.pi / 2, -np.pi, 3 * np.pi / 2, 1e-8, -1e-300]])
    got = _run(exe, "s", xs)
    for x, (s, c) in zip(xs, got):
        ms, mc = mp.sin(mp.mpf(float(x))), mp.cos(mp.mpf(float(x)))
        # absolute error against 1 (the scale of sin and cos) stays at a few ulp
        assert abs(s - float(ms)) <= 4 * 2.0 ** -52 * max(1.0, abs(x) * 2.0 ** -20) + 1e-300
        assert abs(c - float(mc)) <= 4 * 2.0 ** -52 * max(1.0, abs(x) * 2.0 ** -20)


def test_cos_reduced(exe):
    mp.mp.dps = 40
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-4 * np.pi, 4 * np.pi, 400), rng.uniform(-1e4, 1e4, 200),
                         [0.0, np.pi / 2, -np.pi / 2, np.pi, 3 * np.pi / 2, 1e-9]])
    got = _run(exe, "c", xs)
    for x, (c,) in zip(xs, got):
        assert abs(c - float(mp.cos(mp.mpf(float(x))))) <= 4 * 2.0 ** -52 * max(1.0, abs(x) * 2.0 ** -20)


def test_reduce_2pi(exe):
    """x - 2 pi rint(x / 2 pi) to a few ulp of pi for |x| up to 6e6."""
    mp.mp.dps = 50
    rng = np.random.default_rng(2)
    xs = np.concatenate([rng.uniform(-10, 10, 200), rng.uniform(-6e6, 6e6, 200), [0.0, np.pi, -np.pi]])
    got = _run(exe, "r", xs)
    for x, (r,) in zip(xs, got):
        X = mp.mpf(float(x))
        n = mp.nint(X / (2 * mp.pi))
        want = X - 2 * mp.pi * n
        assert abs(r - float(want)) <= 8 * 2.0 ** -52 * 4, (x, r, want)


def test_exp_split(exe):
    mp.mp.dps = 40
    xs = np.concatenate([-np.logspace(-12, np.log10(700.0), 300), np.logspace(-12, np.log10(700.0), 300),
                         [0.0, -0.5, 0.5, -0.34657359, 0.34657359]])
    got = _run(exe, "e", xs)
    for x, (t, m) in zip(xs, got):
        et, em = mp.exp(mp.mpf(float(x))), mp.expm1(mp.mpf(float(x)))
        assert _ulp_err(t, et) <= 3
        assert _ulp_err(m, em) <= 4


@pytest.mark.parametrize("kind", ["fermi", "bose"])
def test_leaf_pair_and_derivative(exe, kind):
    """f(y), f(-y) = 1 - f(y) and f'(y) = -f(y) f(-y) to a few ulp relative, from
    y = 1e-10 (next to the Bose pole) out to |y| = 700."""
    mp.mp.dps = 40
    mag = np.logspace(-10, np.log10(690.0), 250)   # arguments are clamped at 700
    ys = np.concatenate([mag, -mag])
    got = _run(exe, kind[0], ys)
    sig = 1 if kind == "fermi" else -1
    for y, (f, fm, df) in zip(ys, got):
        Y = mp.mpf(float(y))
        ef = 1 / (sig * mp.exp(Y) + 1)
        efm = 1 / (sig * mp.exp(-Y) + 1)
        assert _ulp_err(f, ef) <= 8, (y, f, ef)
        assert _ulp_err(fm, efm) <= 8, (y, fm, efm)
        assert _ulp_err(df, -ef * efm) <= 12, (y, df)


@pytest.mark.parametrize("kind", ["fermi", "bose"])
def test_leaf_and_slope_equal_the_pair(exe, kind):
    """leaf_and_slope gives the leaf_pair value and exactly -f(y) f(-y)."""
    mag = np.logspace(-10, np.log10(690.0), 200)
    ys = np.concatenate([mag, -mag, [0.0]] if kind == "fermi" else [mag, -mag])   # the Bose pole at 0 aside
    pair = _run(exe, kind[0], ys)
    slope = _run(exe, "u" if kind == "fermi" else "v", ys)
    for (f, fm, _), (f2, dv) in zip(pair, slope):
        assert f2 == f and dv == -(f * fm)


@pytest.mark.parametrize("kind", ["fermi", "bose"])
def test_leaf_at_complex_arguments(exe, kind):
    """1/(sigma e^y + 1) at complex y to a few ulp relative: |Re y| from 1e-10
    to 690, Im y up to 60, next to the Bose pole at 0, away from the Fermi
    poles at i pi (2n+1)."""
    mp.mp.dps = 40
    rng = np.random.default_rng(62)
    mag = np.logspace(-10, np.log10(690.0), 120)
    yr = np.concatenate([mag, -mag, rng.uniform(-5, 5, 200), [0.0, 0.0, 1e-9, -1e-9]])
    yi = np.concatenate([rng.uniform(-3, 3, 240), rng.uniform(-60, 60, 200), [0.3, -2.0, 1e-9, -2e-9]])
    sig = 1 if kind == "fermi" else -1
    if sig == 1:   # keep a distance of 0.05 from the Fermi poles
        near = np.abs(yr) < 0.05
        d = np.abs((yi / np.pi - 1) / 2 - np.round((yi / np.pi - 1) / 2)) * 2 * np.pi
        keep = ~(near & (d < 0.05))
        yr, yi = yr[keep], yi[keep]
    res = subprocess.run([exe, "F" if sig == 1 else "B"],
                         input="\n".join(f"{float(a)!r} {float(b)!r}" for a, b in zip(yr, yi)),
                         capture_output=True, text=True, check=True)
    got = np.array([[float(v) for v in l.split()] for l in res.stdout.splitlines()])
    assert got.shape == (len(yr), 2)
    for a, b, (fr, fi) in zip(yr, yi, got):
        Y = mp.mpc(float(a), float(b))
        want = 1 / (sig * mp.exp(Y) + 1)
        err = abs(mp.mpc(fr, fi) - want)
        # relative to |f|; the reduction of Im y modulo 2 pi costs up to |Im y| / 4 ulp
        bound = (8 + abs(b) / 4) * 2.0 ** -52 * abs(want)
        assert err <= bound + 1e-300, (a, b, fr, fi, complex(want))


def test_device_philox_matches_oracle_and_known_answers(exe):
    from oracle.mc import draw_momenta, philox4x32
    rng = np.random.default_rng(61)
    rows = [[0, 0, 0, 0, 0, 0], [2 ** 32 - 1] * 6,
            [0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344, 0xa4093822, 0x299f31d0]]
    rows += rng.integers(0, 2 ** 32, size=(40, 6)).tolist()
    res = subprocess.run([exe, "p"], input="\n".join(" ".join(str(int(x)) for x in r) for r in rows),
                         capture_output=True, text=True, check=True)
    out = [l.split() for l in res.stdout.splitlines()]
    assert len(out) == len(rows)
    for r, o in zip(rows, out):
        want = philox4x32(r[:4], r[4:])
        assert [int(x) for x in o[:4]] == want
        assert [float(x) for x in o[4:]] == [((w + 0.5) * 2.0 ** -32 - 0.5) * 2 * np.pi for w in want]
    assert [int(x) for x in out[0][:4]] == [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    # the sample layout of oracle.mc: sample 5, seed 9 -> counter (5, 0, b, 0), key (9, 0)
    k = draw_momenta(5, 1, 8, seed=9)[0]
    res = subprocess.run([exe, "p"], input="5 0 0 0 9 0\n5 0 1 0 9 0\n", capture_output=True, text=True,
                         check=True)
    dev = [float(x) for l in res.stdout.splitlines() for x in l.split()[4:]]
    assert dev == k.tolist()
