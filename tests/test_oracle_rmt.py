"""Oracle pins from random-matrix theory (Section 2, eq. mplaw-ev / mplaw-sv, Figs. 1-2)
and statistical checks of the synthetic workloads the oracle is used on."""
import json
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.stats

import oracle
import synth
from conftest import GOLDEN


def _paper():
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("rho", [0.5, 1.5, 1.86, 3.0])
def test_mp_densities_have_unit_mass(rho):
    lm = (1 - np.sqrt(rho)) ** 2
    lp = (1 + np.sqrt(rho)) ** 2
    m1, _ = scipy.integrate.quad(lambda x: oracle.mp_eigen_density(np.array([x]), rho)[0],
                                 lm, lp, limit=200)
    sm, sp = oracle.mp_singular_edges(rho)
    m2, _ = scipy.integrate.quad(lambda x: oracle.mp_singular_density(np.array([x]), rho)[0],
                                 sm, sp, limit=200)
    assert abs(m1 - 1.0) < 1e-6 and abs(m2 - 1.0) < 1e-6
    # the eigenvalue edges are the squared singular-value edges
    assert abs(sp ** 2 - lp) < 1e-12 and abs(sm ** 2 - lm) < 1e-12


def test_fig1_printed_outlier_threshold():
    f1 = _paper()["fig1_mp_outlier_threshold"]
    _, sp = oracle.mp_singular_edges(f1["rho"])
    # singular values of the unnormalised matrix: scale by sqrt(smaller dimension)
    thr = f1["factor"] * sp * np.sqrt(min(f1["rows"], f1["cols"]))
    assert abs(thr - f1["printed"]) <= f1["printed_resolution"]
    naive = _paper()["fig1_rho_expected"]
    assert round(max(f1["rows"], f1["cols"]) / min(f1["rows"], f1["cols"]), 2) == naive["printed"]


def test_fig2_gaussian_sample_follows_mp():
    f2 = _paper()["fig2_mp_sample"]
    rows, cols, rho = f2["rows"], f2["cols"], f2["rho"]
    X = np.random.default_rng(12).standard_normal((rows, cols))
    sv = np.linalg.svd(X / np.sqrt(cols), compute_uv=False)
    sm, sp = oracle.mp_singular_edges(rho)
    grid = np.linspace(sm, sp, 20001)
    pdf = oracle.mp_singular_density(grid, rho)
    cdf = np.concatenate([[0.0], np.cumsum((pdf[1:] + pdf[:-1]) * 0.5 * np.diff(grid))])
    cdf /= cdf[-1]
    ks = scipy.stats.kstest(sv, lambda x: np.interp(x, grid, cdf))
    assert ks.statistic < 0.03
    assert abs(sv.max() - sp) < 0.05 * sp


def test_null_genotype_bulk_edge():
    # unstructured genotypes: top singular value at the noise edge sqrt(1-m)(sqrt n + sqrt p)
    n, p, miss = 400, 3000, 0.01
    rng = np.random.default_rng(4)
    f = rng.uniform(0.05, 0.5, size=p)
    packed = synth.generate(n, p, 99, f, miss_rate=miss)
    op = oracle.PackedOperator(packed, n, p)
    res = oracle.gkl_svd(op, 3, tol=1e-10, v0=synth.start_vector(p, 4))
    edge = synth.mp_edge(n, p, miss)
    assert abs(res.sigma[0] / edge - 1.0) < 0.03


def test_planted_spikes_follow_bbp():
    # rank-3 spikes in the unclipped regime (f in [0.2, 0.5], small per-entry
    # amplitude): outliers at the rectangular BBP location, +-5%
    n, p, miss = 2000, 20000, 0.01
    rng = np.random.default_rng(8)
    f = rng.uniform(0.2, 0.5, size=p)
    ratios = np.array([5.0, 3.0, 2.0])
    c = n / p
    theta = np.array([synth.bbp_theta(r, c) for r in ratios])
    t = theta * np.sqrt(p / (1.0 - miss))
    x = rng.choice([-1.0, 1.0], size=(3, n)) / np.sqrt(n)
    y = rng.choice([-1.0, 1.0], size=(3, p)) / np.sqrt(p)
    d = np.sqrt(2.0 * f * (1.0 - f))
    packed = synth.generate(n, p, 31, f, (x * t[:, None]).T, y * (d / 2.0)[None, :],
                            miss_rate=miss)
    res = oracle.gkl_svd(oracle.PackedOperator(packed, n, p), 4, tol=1e-10,
                         v0=synth.start_vector(p, 6))
    edge = synth.mp_edge(n, p, miss)
    assert np.all(np.abs(res.sigma[:3] / (ratios * edge) - 1.0) < 0.05)
    assert res.sigma[3] < 1.05 * edge


def test_spiked_workload_separates_ten_outliers():
    # the full spiked recipe at a small shape: all ten planted spikes leave the bulk
    g = synth.config("c5", n=1500, p=15000)
    op = oracle.PackedOperator(g.packed, g.n, g.p)
    res = oracle.gkl_svd(op, 10, tol=1e-10, v0=synth.start_vector(g.p, 5))
    assert res.sigma[9] > 1.1 * g.meta["edge"]


def test_algorithm1_model_spectrum():
    # the paper's model (Algorithm 1) at a small size: a handful of large outliers
    # and zero singular values from duplicated rows
    rows, cols = 300, 600
    M = synth.algorithm1_codes(rows, cols, r=10, nsignal=rows * cols, rkins=0.05, seed=3)
    n_dup = rows - np.unique(M, axis=0).shape[0]
    packed = synth.pack_codes(M)
    st = oracle.column_stats(rows, *oracle.counts(packed, rows, cols))
    A = oracle.dense_matrix(oracle.decode(packed, rows, cols), st.mean, st.inv_sd)
    s = np.linalg.svd(A, compute_uv=False)
    assert n_dup >= 5
    assert np.sum(s < 1e-9 * s[0]) >= n_dup
    res = oracle.gkl_svd(oracle.DenseOperator(A), 10, tol=1e-12, v0=synth.start_vector(cols, 2))
    assert np.all(np.abs(res.sigma - s[:10]) <= 1e-10 * s[0])
