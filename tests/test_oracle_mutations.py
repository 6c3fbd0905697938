"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (a dropped
coordinate term, a reversed tie-break, an exclusive radius, 1/(n-1), a
wrong mean divisor, the largest eigenvector, a flipped regulariser sign, a
wrong Jacobi rotation sign, a wrong validity threshold; in the weighted
covariance a wrong kernel exponent, a flipped weight sign, an unnormalised
mean, an unweighted sum, a wrong reference point; in the GICP system a
Jacobian or residual sign, a missing inverse or transpose, a dropped
covariance, a tie or radius slip in the correspondences), compiles it on the
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
from tests import test_oracle_gicp as gpins
from tests import test_oracle_voxel as vpins
from tests import test_oracle_walls as wlpins

SRC = os.path.join(os.path.dirname(oracle.__file__), "lkc_oracle.c")

MUTATIONS = {
    "dropped_dz": ("dx * dx + dy * dy + dz * dz;\n            if (!(d <= jb->r2))",
                   "dx * dx + dy * dy;\n            if (!(d <= jb->r2))"),
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

# planted mistakes in the GICP correspondence search and Gauss-Newton system
GICP_MUTATIONS = {
    "jacobian_skew_sign": ("{0.0, -p[2], p[1], -1.0, 0.0, 0.0}",
                           "{0.0, p[2], -p[1], -1.0, 0.0, 0.0}"),
    "residual_sign": ("d[r] = (double)tgt[3 * (int64_t)j + r] - p[r];",
                      "d[r] = p[r] - (double)tgt[3 * (int64_t)j + r];"),
    "no_inverse": ("if (!inv3_adjugate(M, W))", "if (!inv3_adjugate(M, W) || !memcpy(W, M, sizeof W))"),
    "rotation_not_transposed": ("s += RC[3 * r + a] * R[3 * c + a];",
                                "s += RC[3 * r + a] * R[3 * a + c];"),
    "target_cov_dropped": ("M[3 * r + c] = (double)tgt_cov[9 * (int64_t)j + 3 * r + c] + s;",
                           "M[3 * r + c] = s;"),
    "corr_later_tie": ("(d < bd || (d == bd && j < best))", "(d <= bd)"),
    "corr_radius_exclusive": ("if (d <= jb->r2 && (d < bd", "if (d < jb->r2 && (d < bd"),
    "b_sign": ("b[r] += J[0][r] * Wd[0]", "b[r] -= J[0][r] * Wd[0]"),
    "adjugate_entry": ("inv[5] = (M[2] * M[3] - M[0] * M[5]) / det;",
                       "inv[5] = (M[0] * M[5] - M[2] * M[3]) / det;"),
}

GICP_PINS = [getattr(gpins, n) for n in dir(gpins) if n.startswith("test_")]

# planted mistakes in the voxel filter and the submap window
VOXEL_MUTATIONS = {
    "voxel_order_x_first": ("for (int d = 2; d >= 0; --d) {\n        if (x->v[d] != y->v[d])",
                            "for (int d = 0; d < 3; ++d) {\n        if (x->v[d] != y->v[d])"),
    "voxel_trunc": ("const double f = floor((double)q);", "const double f = trunc((double)q);"),
    "voxel_mean_divisor": ("s[d] / (double)(b - a);", "s[d] / (double)(b - a + 1);"),
    "voxel_reciprocal": ("const float q = (p[d] - origin[d]) / leaf;",
                         "const float q = (p[d] - origin[d]) * (1.0f / leaf);"),
    "submap_exclusive": ("if (d2 <= r2)\n            out[m++]", "if (d2 < r2)\n            out[m++]"),
    "submap_dropped_z": ("const double d2 = dx * dx + dy * dy + dz * dz;\n        if (d2 <= r2)",
                         "const double d2 = dx * dx + dy * dy;\n        if (d2 <= r2)"),
}

VOXEL_PINS = [getattr(vpins, n) for n in dir(vpins) if n.startswith("test_")]

# planted mistakes in the z-vote filter and the clustering
WALL_MUTATIONS = {
    "zvote_trunc": ("r[m].u = (int64_t)floor((double)(p[0] / g));",
                    "r[m].u = (int64_t)trunc((double)(p[0] / g));"),
    "zvote_v_from_x": ("r[m].v = (int64_t)floor((double)(p[1] / g));",
                       "r[m].v = (int64_t)floor((double)(p[0] / g));"),
    "zvote_strict": ("keep[r[c].i] = (uint8_t)((b - a) >= tau);",
                     "keep[r[c].i] = (uint8_t)((b - a) > tau);"),
    "cluster_exclusive": ("if (d2 <= e2) {", "if (d2 < e2) {"),
    "cluster_max_label": ("par[a > b ? a : b] = a < b ? a : b;",
                          "par[a < b ? a : b] = a > b ? a : b;"),
    "cluster_dropped_dz": ("const double d2 = dx * dx + dy * dy + dz * dz;\n            if (d2 <= e2)",
                           "const double d2 = dx * dx + dy * dy;\n            if (d2 <= e2)"),
}

WALL_PINS = [getattr(wlpins, n) for n in dir(wlpins) if n.startswith("test_")]


def _call(pin):
    marks = getattr(pin, "pytestmark", [])
    params = [m for m in marks if m.name == "parametrize"]
    if not params:
        return pin()
    names = [a.strip() for a in params[0].args[0].split(",")]
    for vals in params[0].args[1]:
        pin(**dict(zip(names, vals if len(names) > 1 else (vals,))))


def test_unmutated_source_passes_the_pins():
    for pin in PINS + WEIGHTED_PINS + GICP_PINS + VOXEL_PINS + WALL_PINS:
        _call(pin)


GROUPS = [(MUTATIONS, PINS), (WEIGHTED_MUTATIONS, WEIGHTED_PINS), (GICP_MUTATIONS, GICP_PINS),
          (VOXEL_MUTATIONS, VOXEL_PINS), (WALL_MUTATIONS, WALL_PINS)]


@pytest.mark.parametrize("name", [n for muts, _ in GROUPS for n in sorted(muts)])
def test_pins_catch_planted_mistake(name, tmp_path):
    muts, pins_for = next((m, p) for m, p in GROUPS if name in m)
    old, new = muts[name]
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
