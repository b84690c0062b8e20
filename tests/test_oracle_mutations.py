"""Planted mistakes in the FP64 oracle, on the CPU: each plausible slip in its arithmetic (a dropped term or factor,
a flipped sign, a shifted index, the wrong channel, an edge case, a swapped argument) makes at least one pin of
``test_oracle_pins.py`` fail, so those pins would have caught it.

Each case copies ``oracle/wt_oracle.c``, replaces one fragment of it, builds the copy with gcc into a temporary
library and runs the named pins against a fresh instance of the oracle module bound to that library. Nothing here
touches the oracle that the other tests use.
"""
import importlib.util
import os
import subprocess

import pytest

import test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "wt_oracle.c")
pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

# (what the mistake is, text replaced, replacement, which occurrence, pins expected to catch it)
MUTATIONS = [
    ("scaling coefficient without its 1 - x factor", "coef[0] += a[i] * (1.0 - x[i]);", "coef[0] += a[i];", 0,
     [("test_p2_closed_forms_match_inner_products", {"seed": 0})]),
    ("wavelet coefficients with the wrong sign", "double X = -a[i] * orc_Psi(n, k, x[i]);",
     "double X = a[i] * orc_Psi(n, k, x[i]);", 0, [("test_p4_sign_of_coefficients", {})]),
    ("interpolation from cell j instead of j - 1", "double lo = (j == 0) ? 0.0 : cells[j - 1];",
     "double lo = cells[j];", 0, [("test_p1_worked_example_single_layer", {})]),
    ("background weighted by the first channel's transmittance", "int c = (C == 3) ? q : 0;", "int c = 0;", 0,
     [("test_p8_grid_depths_three_channels", {})]),
    ("brute-force A-buffer lets equal depths occlude",
     "if (clamp_depth(depth[order[q]]) < xr) prod", "if (clamp_depth(depth[order[q]]) <= xr) prod", 0,
     [("test_abuffer_sorted_equals_brute_force", {})]),
    ("shared-exponent mantissas truncated", "uint32_t m = (uint32_t)floor(ldexp(v[q], 24 - es) + 0.5);",
     "uint32_t m = (uint32_t)floor(ldexp(v[q], 24 - es));", 0, [("test_e5b9g9r9_hand_worked", {})]),
    ("depth bounds map divides by zmax", "(xs[r] - lo) / (hi - lo)", "(xs[r] - lo) / hi", 0,
     [("test_tight_depth_two_layers_are_exact", {"channels": 1})]),
    ("gradient drops the background term", "double inner = bg[q] * T;", "double inner = 0.0;", 0,
     [("test_p14_backward_matches_finite_differences", {"channels": 1})]),
    ("gradient without the chain factor of the absorbance", "direct + dLda / (1.0 - au)", "direct + dLda", 0,
     [("test_p14_backward_matches_finite_differences", {"channels": 1})]),
    ("one-pass shading ignores the reprojection map", "const uint64_t src = prev_pixel ? prev_pixel[p] : (uint64_t)p;",
     "const uint64_t src = (uint64_t)p;", 0, [("test_shade_prev_single_previous_layer_closed_form", {"channels": 1})]),
    ("one-pass shading without the previous visibility", "double v = exp(-orc_reconstruct((int)rank, ce, xs[r]));",
     "double v = 1.0;", 1, [("test_shade_prev_single_previous_layer_closed_form", {"channels": 1})]),
    ("one-pass background from the first channel", "int c = (C == 3) ? q : 0;", "int c = 0;", 1,
     [("test_shade_prev_without_history_sees_nothing_in_front", {"channels": 3})]),
    ("chromatic taps displaced the wrong way", "double s = 1.0 + dispersion", "double s = 1.0 - dispersion", 0,
     [("test_chromatic_linear_background_closed_form", {"taps": 5, "disp": 0.5})]),
    ("chromatic taps from the pixel corner, not its centre",
     "double cx = (double)(p % width) + 0.5, cy = (double)(p / width) + 0.5;",
     "double cx = (double)(p % width), cy = (double)(p / width);", 0,
     [("test_chromatic_zero_offset_reads_the_pixel", {"channels": 1})]),
    ("chromatic weights not normalised", "* num[q] / den[q];", "* num[q];", 0,
     [("test_chromatic_uniform_background_is_the_plain_composite", {})]),
    ("red and blue spectral weights swapped",
     "w[0] = smoothstep_formula(0.5, 1.0 / 3.0, t);\n  w[2] = smoothstep_formula(0.5, 2.0 / 3.0, t);",
     "w[2] = smoothstep_formula(0.5, 1.0 / 3.0, t);\n  w[0] = smoothstep_formula(0.5, 2.0 / 3.0, t);", 0,
     [("test_spectral_weights_golden", {})]),
]


def _mutant(tmp_path, old, new, occurrence):
    src = open(SRC).read()
    at = -1
    for _ in range(occurrence + 1):
        at = src.find(old, at + 1)
        assert at >= 0, "the oracle no longer contains the text this case replaces: %r" % old
    c = tmp_path / "mutant.c"
    c.write_text(src[:at] + new + src[at + len(old):])
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", str(so), str(c), "-lm"])
    spec = importlib.util.spec_from_file_location("oracle_mutant", os.path.join(ROOT, "oracle", "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._LIB = str(so)
    mod._lib = None
    return mod


@pytest.mark.parametrize("what,old,new,occurrence,checks", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, what, old, new, occurrence, checks):
    mod = _mutant(tmp_path, old, new, occurrence)
    caught = []
    for name, kwargs in checks:
        try:
            getattr(pins, name)(mod, **kwargs)
        except (AssertionError, RuntimeError, ValueError) as e:
            caught.append((name, type(e).__name__))
    assert caught, "no pin caught the planted mistake: %s" % what


def test_unmutated_copy_passes_the_same_pins(tmp_path):
    """The harness itself: a copy with no change passes every pin the cases use."""
    mod = _mutant(tmp_path, "coef[0] += a[i] * (1.0 - x[i]);", "coef[0] += a[i] * (1.0 - x[i]);", 0)
    seen = set()
    for _, _, _, _, checks in MUTATIONS:
        for name, kwargs in checks:
            key = (name, tuple(sorted(kwargs.items())))
            if key not in seen:
                seen.add(key)
                getattr(pins, name)(mod, **kwargs)
