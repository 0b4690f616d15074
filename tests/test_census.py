"""The operation census evaluates a correct right-hand side: its formulas give
the oracle's values (so the flop counts used for the roofline belong to a
correct evaluation of Hamilton's equations)."""
import numpy as np
import pytest

from paper_2605_05635_amd import census
from paper_2605_05635_amd import workloads as W


@pytest.mark.parametrize("metric,halo", [("kerr", (0.0, 0.0)), ("einasto", (0.2, 0.0)),
                                         ("cnfw", (0.03, 7.0))])
def test_census_formulas_match_oracle_rhs(orc, metric, halo):
    img = W.image(metric=metric, spin=0.7, halo=halo)
    c = dict(chi=0.7, chi2=0.49, inv_lam=1 / halo[0] if halo[0] else 0.0, lam_c=halo[1] or 1.0,
             inv_lam_c=1 / (halo[1] or 1.0),
             eta_lc=halo[0] * halo[1])
    rng = np.random.default_rng(2)
    for _ in range(20):
        R, th = rng.uniform(2.2, 60), rng.uniform(0.2, 2.9)
        E, L, pR, pth = rng.uniform(0.8, 1.2), rng.uniform(-4, 4), rng.normal(), rng.normal()
        got = [float(v) for v in census.rhs(metric, c, census.Num(E), census.Num(L),
                                             census.Num(R), census.Num(th), census.Num(pR),
                                             census.Num(pth))]
        want = orc.rhs(img, E, L, [0, R, th, 0, pR, pth])
        assert np.allclose(got, want, rtol=1e-11, atol=1e-13)


def test_census_counts_are_positive_and_ordered():
    k, e, c = (census.flops_rhs(m) for m in ("kerr", "einasto", "cnfw"))
    assert 50 < k < e < c < 200
    assert 250 < census.flops_step_overhead() < 450
    assert 150 < census.flops_crossing() < 400
    ke, ee, ce = (census.flops_emission(m) for m in ("kerr", "einasto", "cnfw"))
    assert 20 < ke < ee < ce < 120


def test_thick_source_count():
    from paper_2605_05635_amd import census
    for m in ("kerr", "einasto", "cnfw"):
        # the source adds the emissivity's exponentials and the local metric to
        # the Keplerian redshift of the thin disc
        assert census.flops_emission(m) < census.flops_thick_source(m) < 3 * census.flops_emission(m)
