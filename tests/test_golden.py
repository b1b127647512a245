"""The fixtures of printed values (tests/golden/) and the workload constants that the
paper's cases take from them: the density ratios of Sec. 3.2.1 and the confinement
factor of Eq. (34), which the sedimentation workloads use to set gravity (Eq. (35))."""
import math

from golden import printed

from paper_1905_05110_amd import workloads as W


def test_every_fixture_value_cites_its_passage():
    vals = printed()
    assert len(vals) >= 10
    for name, (v, cite) in vals.items():
        assert math.isfinite(v), name
        assert "Sec. 3" in cite, (name, cite)


def test_density_ratios_are_the_printed_list():
    vals = printed()
    ratios = tuple(vals["density_ratio_settling_%d" % i][0] for i in range(1, 7))
    assert ratios == tuple(W.PAPER_DENSITY_RATIOS)


def test_confinement_factor_uses_the_printed_coefficients():
    vals = printed()
    c = {k: vals["kappa_coeff_%d" % k][0] for k in (0, 2, 4, 6, 8)}
    for Ht in (5.0, 12.5, 32.0, 100.0):
        poly = math.log(Ht) + c[0] + sum(c[k] * Ht ** -k for k in (2, 4, 6, 8))
        assert abs(W.confinement_kappa(Ht) - 1.0 / poly) <= 1e-15 / poly
    # the 1024 x 4096 box (H/D = 32) of the sedimentation workload
    assert abs(W.confinement_kappa(32.0) - 0.39189) < 5e-6
