"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (a dropped
coordinate term, a reversed tie-break, an exclusive radius, 1/(n-1), a
wrong mean divisor, the largest eigenvector, a flipped regulariser sign, a
wrong Jacobi rotation sign, a wrong validity threshold; in the weighted
covariance a wrong kernel exponent, a flipped weight sign, an unnormalised
mean, an unweighted sum, a wrong reference point), compiles it on the
CPU, swaps it in for the real oracle and runs the pin tests: at least one
must fail.  The real oracle is restored afterwards.
"""
import ctypes
import os
import subprocess

import pytest

from oracle import oracle
from tests import test_oracle as pins
from tests import test_oracle_weighted as wpins

SRC = os.path.join(os.path.dirname(oracle.__file__), "lkc_oracle.c")

MUTATIONS = {
    "dropped_dz": ("dx * dx + dy * dy + dz * dz", "dx * dx + dy * dy"),
    "tiebreak_reversed": ("(da == db && ia < ib)", "(da == db && ia > ib)"),
    "radius_exclusive": ("if (!(d <= jb->r2))", "if (!(d < jb->r2))"),
    "cov_n_minus_1": ("c[e] /= (double)n;", "c[e] /= (double)(n - 1);"),
    "mean_divisor": ("mu[a] /= (double)n;", "mu[a] /= (double)(n + 1);"),
    "largest_eigvec": ("V[3 * r + 0] * V[3 * cc + 0]", "V[3 * r + 2] * V[3 * cc + 2]"),
    "reg_sign": ("eye - (1.0 - jb->eps)", "eye + (1.0 - jb->eps)"),
    "rotation_sign": ("a[r][p] = c * arp - s * arq;", "a[r][p] = c * arp + s * arq;"),
    "valid_threshold": ("const int ok = (n >= 3);", "const int ok = (n >= 2);"),
}

PINS = [
    lambda: [pins.test_knn_matches_exhaustive_python(s, r) for s in range(3)
             for r in (float("inf"), 0.7)],
    pins.test_knn_1d_lattice_windows_and_tiebreak,
    pins.test_knn_2d_3d_lattice_ties_and_dropped_terms,
    pins.test_knn_radius_is_inclusive_and_caps_count,
    pins.test_cov_1d_lattice_closed_form,
    pins.test_cov_matches_numpy_cov_bias_and_twin,
    pins.test_cov_invariants,
    pins.test_cov_small_counts,
    pins.test_jacobi_matches_eigh,
    pins.test_regulariser_eigenvalues_and_closed_form,
    pins.test_noisy_plane_and_wall_normals,
]


# planted mistakes in the kernel-descriptor weighted covariance
WEIGHTED_MUTATIONS = {
    "rbf_divides": ("kind == 1 ? d2 * sigma", "kind == 1 ? d2 / sigma"),
    "gauss_no_half": ("d2 / (2.0 * sigma * sigma)", "d2 / (sigma * sigma)"),
    "laplacian_squared": (": sqrt(d2) / sigma", ": d2 / sigma"),
    "weight_sign": ("const double w = exp(-(e[j] - emin));\n                sw += w;",
                    "const double w = exp(+(e[j] - emin));\n                sw += w;"),
    "mean_unnormalised": ("mu[a] /= sw;", "mu[a] /= (double)m;"),
    "cov_unweighted": ("c[3 * r + cc] += w * d[r] * d[cc];", "c[3 * r + cc] += d[r] * d[cc];"),
    "reference_first_neighbour": ("ref[a] = queries ? (double)queries[3 * qi + a]",
                                  "ref[a] = 0 ? (double)queries[3 * qi + a]"),
    "weighted_valid": ("const int ok = (m >= 3);", "const int ok = (m >= 1);"),
}

WEIGHTED_PINS = [getattr(wpins, n) for n in dir(wpins) if n.startswith("test_")]


def _call(pin):
    marks = getattr(pin, "pytestmark", [])
    params = [m for m in marks if m.name == "parametrize"]
    if not params:
        return pin()
    names = [a.strip() for a in params[0].args[0].split(",")]
    for vals in params[0].args[1]:
        pin(**dict(zip(names, vals if len(names) > 1 else (vals,))))


def test_unmutated_source_passes_the_pins():
    for pin in PINS + WEIGHTED_PINS:
        _call(pin)


@pytest.mark.parametrize("name", sorted(MUTATIONS) + sorted(WEIGHTED_MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS.get(name) or WEIGHTED_MUTATIONS[name]
    pins_for = PINS if name in MUTATIONS else WEIGHTED_PINS
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so),
                           str(mut), "-lpthread", "-lm"])
    real = oracle._load()
    oracle._lib = oracle.configure(ctypes.CDLL(str(so)))
    failed = []
    try:
        for pin in pins_for:
            try:
                _call(pin)
            except (AssertionError, ValueError):
                failed.append(pin)
    finally:
        oracle._lib = real
    assert failed, f"no pin caught the planted mistake {name}"
