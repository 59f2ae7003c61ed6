"""Mutation check of the oracle's pins: each plausible mistake below is planted in a
copy of oracle/crb_ref.c (on the CPU), compiled, and must fail at least one pin.
A surviving mutant would mean the pins cannot tell that mistake from the method."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import ref
import tests.test_oracle_pins as P
import tests.test_oracle_sources as SRCP

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "crb_ref.c")

# (name, text to find (must occur exactly once), replacement)
MUTANTS = [
    ("laplacian centre weight", "double v = 4.0 * c - u - d - l - r;",
     "double v = 3.0 * c - u - d - l - r;"),
    ("laplacian neighbour row", "double d = J2[(size_t)clampi(Y + 1, H2) * W2 + X];",
     "double d = J2[(size_t)clampi(Y - 1, H2) * W2 + X];"),
    ("no negative clip", "L2[(size_t)Y * W2 + X] = v > 0.0 ? v : 0.0;",
     "L2[(size_t)Y * W2 + X] = v;"),
    ("rebin sum not mean", "(a + b + c + d) / 4.0;", "(a + b + c + d) / 2.0;"),
    ("gain missing in noise", "sqrt(p->gain * m + p->readnoise * p->readnoise) / p->gain;",
     "sqrt(m + p->readnoise * p->readnoise) / p->gain;"),
    ("no division by gain", "sqrt(p->gain * m + p->readnoise * p->readnoise) / p->gain;",
     "sqrt(p->gain * m + p->readnoise * p->readnoise);"),
    ("read noise not squared", "p->readnoise * p->readnoise) / p->gain;",
     "p->readnoise) / p->gain;"),
    ("noise floor", "m = 1e-4;", "m = 1.0;"),
    ("sky ignored", "double m = m5[i] + p->sky;", "double m = m5[i];"),
    ("subsampling factor", "S[i] = Lp[i] / (2.0 * N[i]);", "S[i] = Lp[i] / N[i];"),
    ("S' sign", "Sp[i] = S[i] - mS[i];", "Sp[i] = S[i] + mS[i];"),
    ("S' without med5", "Sp[i] = S[i] - mS[i];", "Sp[i] = S[i];"),
    ("med7 radius", "crb_ref_median_filter(m3, H, W, 3, m7)", "crb_ref_median_filter(m3, H, W, 2, m7)"),
    ("fine structure sign", "double f = (m3[i] - m7[i]) / N[i];", "double f = (m7[i] - m3[i]) / N[i];"),
    ("F not normalised", "double f = (m3[i] - m7[i]) / N[i];", "double f = (m3[i] - m7[i]);"),
    ("F floor", "Fh[i] = f < 0.01 ? 0.01 : f;", "Fh[i] = f < 0.1 ? 0.1 : f;"),
    ("objlim ignored", "A[i] = (Sp[i] > p->sigclip && Sp[i] / Fh[i] > p->objlim) ? 1 : 0;",
     "A[i] = (Sp[i] > p->sigclip) ? 1 : 0;"),
    ("non-strict threshold", "A[i] = (Sp[i] > p->sigclip && Sp[i] / Fh[i] > p->objlim) ? 1 : 0;",
     "A[i] = (Sp[i] >= p->sigclip && Sp[i] / Fh[i] > p->objlim) ? 1 : 0;"),
    ("grow 1 gated low", "G1[i] = (D[i] && Sp[i] > p->sigclip) ? 1 : 0;",
     "G1[i] = (D[i] && Sp[i] > lowlim) ? 1 : 0;"),
    ("grow 2 gated high", "G2[i] = (D[i] && Sp[i] > lowlim) ? 1 : 0;",
     "G2[i] = (D[i] && Sp[i] > p->sigclip) ? 1 : 0;"),
    ("one grow stage", "dilate3(G1, H, W, D);", "memcpy(D, G1, n);"),
    ("dilation one-sided", "for (int dy = -1; dy <= 1; ++dy)\n                for (int dx = -1; dx <= 1; ++dx)\n                    any |=",
     "for (int dy = 0; dy <= 1; ++dy)\n                for (int dx = 0; dx <= 1; ++dx)\n                    any |="),
    ("count includes old flags", "if (G2[i] && !Mprev[i])", "if (G2[i])"),
    ("mask not cumulative", "M[i] = (Mprev[i] || G2[i]) ? 1 : 0;", "M[i] = G2[i] ? 1 : 0;"),
    ("replacement window 3x3", "for (int dy = -2; dy <= 2; ++dy) {\n                        for (int dx = -2; dx <= 2; ++dx) {",
     "for (int dy = -1; dy <= 1; ++dy) {\n                        for (int dx = -1; dx <= 1; ++dx) {"),
    ("replacement uses flagged", "if (!M[q])\n                                win[cnt++] = J[q];",
     "win[cnt++] = J[q];"),
    ("even median upper", "return 0.5 * (v[n / 2 - 1] + v[n / 2]);", "return v[n / 2];"),
    ("median filter radius", "int k = 2 * r + 1;", "int k = 2 * r + 1; r = r > 1 ? r - 1 : r;"),
    ("early stop test", "if (early_stop && nk == 0)", "if (early_stop && nk <= 1)"),
    ("sources tie order", "return yq > y || (yq == y && xq > x);",
     "return yq < y || (yq == y && xq < x);"),
    ("sources ties always yield", "if (vq == v)\n        return yq > y", "if (vq == v)\n        return 1 || yq > y"),
    ("sources non-strict threshold", "if (!(v > threshold))", "if (!(v >= threshold))"),
    ("sources window short", "for (int yq = y - r; yq <= y + r && peak; ++yq)",
     "for (int yq = y - r + 1; yq <= y + r && peak; ++yq)"),
    ("sources sky kept", "- (double)sky;", "- 0.0 * (double)sky;"),
    ("sources moment sign", "rec.sy = rec.sy + (double)dy * d;", "rec.sy = rec.sy - (double)dy * d;"),
    ("sources aperture half", "for (int dx = -a; dx <= a; ++dx) {", "for (int dx = 0; dx <= a; ++dx) {"),
    ("edge wrap instead of clamp", "static int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }",
     "static int clampi(int i, int n) { return ((i % n) + n) % n; }"),
]


def pin_battery():
    """Fast pins from the pin suite; any AssertionError kills the mutant."""
    P.test_lplus_closed_form_and_scipy()
    P.test_lplus_linear_ramp()
    P.test_constant_images_are_fixed_points()
    P.test_ramp_not_flagged_and_sprime_zero()
    for args in [(7.0, 5.0, 50.0, 0.0), (1.5, 4.0, 200.0, 30.0), (2.0, 0.5, 0.0, 0.0)]:
        P.test_single_pixel_hit_threshold(*args)
    P.test_threshold_is_strict()
    P.test_two_pixel_and_block_tracks()
    for a in [(1.01, 1), (0.99, 0)]:
        P.test_sigfrac_growing(*a)
    for a in [(1.02, 1), (0.98, 0)]:
        P.test_objlim_contrast_on_plateau(*a)
    P.test_replacement_brute_force()
    P.test_replacement_all_flagged_keeps_value()
    P.test_median_filter_matches_scipy_nearest()
    P.test_iteration_matches_scipy_composition()
    P.test_early_stop_neutral_and_invariants()
    P.test_sky_argument_enters_noise_only()
    for args in [(6, 7, 2, 2), (1, 9, 2, 3)]:
        SRCP.test_constant_frame_has_one_source_at_origin(*args)
    for args in [(2, 1, 2), (4, 3, 3)]:
        SRCP.test_brute_force_with_ties(*args)
    SRCP.test_symmetric_star()
    SRCP.test_separation_rule(2)
    SRCP.test_threshold_is_strict_and_plateau_first_pixel()


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="crb_mutants_")
    yield d
    ref.use_library(None)
    shutil.rmtree(d, ignore_errors=True)


def test_unmutated_oracle_passes_the_battery():
    ref.use_library(None)
    pin_battery()


@pytest.mark.parametrize("name,find,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_killed(workdir, name, find, repl):
    src = open(SRC).read()
    assert src.count(find) == 1, f"mutation site not unique: {name}"
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)
    path_c = os.path.join(workdir, f"{tag}.c")
    path_so = os.path.join(workdir, f"{tag}.so")
    with open(path_c, "w") as f:
        f.write(src.replace(find, repl))
    shutil.copy(os.path.join(os.path.dirname(SRC), "crb_ref.h"), workdir)
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", path_so, path_c, "-lm"])
    ref.use_library(path_so)
    try:
        killed = False
        try:
            pin_battery()
        except (AssertionError, ValueError):
            killed = True
        assert killed, f"mutant survived the pins: {name}"
    finally:
        ref.use_library(None)
