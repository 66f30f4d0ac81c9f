"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the C oracle (on the CPU, in a
temporary directory), builds it with gcc, loads it through a fresh copy of
the oracle's Python wrapper and runs the pins of tests/test_oracle_pins.py
against it: at least one pin must fail.  The committed oracle is never
modified.
"""

import importlib.util
import os
import subprocess

import pytest

import tests.test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "svconv_oracle.c")
WRAPPER = os.path.join(ROOT, "oracle", "oracle.py")

MUTATIONS = {
    # correlation instead of convolution (kernel flipped)
    "correlation": [("const int ys = y - v;", "const int ys = y + v;"),
                    ("const int xs = x - u;", "const int xs = x + u;")],
    # x and y exchanged in the spatial terms
    "spatial_xy_swap": [("P[m++] = ipow(xh, i) * ipow(yh, t - i);",
                         "P[m++] = ipow(yh, i) * ipow(xh, t - i);")],
    # coordinates normalised by the frame size instead of size - 1
    "coord_off_by_one": [("return 2.0 * (double)(idx + off) / (double)(frame - 1) - 1.0;",
                          "return 2.0 * (double)(idx + off) / (double)(frame) - 1.0;")],
    # basis monomial with u and v exchanged
    "basis_uv_swap": [("* ipow(u, i) * ipow(v, j);", "* ipow(v, i) * ipow(u, j);")],
    # Gaussian exponent missing its factor 2
    "gaussian_width": [("/ (2.0 * s * s)) * ipow(u, i)", "/ (s * s)) * ipow(u, i)")],
    # bases left unnormalised
    "no_l1_norm": [("for (int q = 0; q < k * k; ++q) B[q] /= l1;",
                    "for (int q = 0; q < k * k; ++q) B[q] /= 1.0;")],
    # coefficient layout read m-major instead of n-major
    "coef_transposed": [("for (int m = 0; m < M; ++m) s += a[n * M + m] * P[m];",
                         "for (int m = 0; m < M; ++m) s += a[m * N + n] * P[m];")],
    # adjoint in a without the spatial term
    "grad_a_drops_P": [("acc[n * M + m] += g * P[m] * T;", "acc[n * M + m] += g * T;")],
    # adjoint in R gathering from the wrong side
    "grad_R_sign": [("const int py = y + v;", "const int py = y - v;"),
                    ("const int px = x + u;", "const int px = x - u;")],
    # normal equations without the spatial term
    "normal_drops_P": [("phi[n * M + m] = P[m] * T[n];", "phi[n * M + m] = T[n];")],
    # Cholesky pivot with the wrong sign of the update
    "cholesky_sign": [("for (int p = 0; p < j; ++p) d -= L[(size_t)j * n + p] * L[(size_t)j * n + p];",
                       "for (int p = 0; p < j; ++p) d += L[(size_t)j * n + p] * L[(size_t)j * n + p];")],
    # last term of the per-pixel kernel sum dropped
    "kernel_drops_last_basis": [("for (int n = 0; n < N; ++n) s += c[n] * basis[(size_t)n * k * k + q];",
                                 "for (int n = 0; n + 1 < N; ++n) s += c[n] * basis[(size_t)n * k * k + q];")],
}


def _pin_calls():
    """(name, callable(orc)) for every pin, parametrised cases spelled out."""
    calls = []
    for name in dir(pins):
        if not name.startswith("test_"):
            continue
        fn = getattr(pins, name)
        if name == "test_regrouped_fft_identity":
            for case in ("c0_full", "c0_crop_frame", "c1_ragged"):
                calls.append((name + "[" + case + "]", lambda o, fn=fn, c=case: fn(o, c)))
        elif name == "test_brute_force_operator_8x8":
            for h in (1, 4, 5):
                calls.append((name + "[%d]" % h, lambda o, fn=fn, h=h: fn(o, h)))
        else:
            calls.append((name, lambda o, fn=fn: fn(o)))
    return calls


def _build_mutant(tmp_path, edits):
    src = open(SRC).read()
    for old, new in edits:
        assert old in src, "mutation anchor not found: %r" % old
        src = src.replace(old, new)
    c_path = tmp_path / "mutant.c"
    c_path.write_text(src)
    so_path = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c99", str(c_path),
                           "-o", str(so_path), "-lm"])
    spec = importlib.util.spec_from_file_location("oracle_mutant_%s" % tmp_path.name, WRAPPER)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._LIB = str(so_path)
    mod._SRC = str(c_path)
    mod._lib = None
    return mod


@pytest.mark.parametrize("mutation", list(MUTATIONS))
def test_pins_catch_planted_mistake(tmp_path, mutation):
    mod = _build_mutant(tmp_path, MUTATIONS[mutation])
    caught = []
    for name, call in _pin_calls():
        try:
            call(mod)
        except (AssertionError, ValueError, Exception) as e:   # noqa: B014 - any failure counts
            if isinstance(e, pytest.skip.Exception):
                raise
            caught.append(name)
    assert caught, "no pin caught the mutation %s" % mutation


def test_unmutated_copy_passes_every_pin(tmp_path):
    # the harness itself: an unmodified copy passes all pins
    mod = _build_mutant(tmp_path, [])
    for name, call in _pin_calls():
        call(mod)
