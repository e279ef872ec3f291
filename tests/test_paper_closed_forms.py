"""The paper's printed closed forms against the values it tabulates."""
from physics_refs import beta_limit, cost_indicator, read_golden, theta_semianalytical


def test_semianalytical_theta_matches_tabulated_curves():
    rows = read_golden("semianalytical_theta.txt")
    assert len(rows) >= 15
    for eps, beta, q, val in rows:
        th = theta_semianalytical(float(beta), float(eps))
        got = th.real if q == "re" else -th.imag
        assert abs(got - float(val)) <= 0.00006, (eps, beta, q, got, val)


def test_cost_indicator_worked_example():
    for chi, s, n, g, G, tol in read_golden("speedup_example.txt"):
        assert abs(cost_indicator(float(chi), float(s), float(n), float(g)) - float(G)) <= float(tol)


def test_beta_limit_brackets_the_paper_grid():
    # the paper's largest beta per eps respects Eq.(betalimit): eps = 0.1 runs
    # reach beta = 100 (< 103.5), eps = 0.075 reaches 150 (< 164.6)
    assert 100 < beta_limit(0.1) < 150
    assert 150 < beta_limit(0.075) < 200


def test_reporting_formula_matches_pinned_reference():
    """The package's semianalytical Theta (used to report the paper's study)
    equals the pinned test reference over the paper's parameter grid."""
    from paper_2006_13631_amd import theory
    from paper_2006_13631_amd.workloads import STUDY_BETA, STUDY_EPS, paper_study_cases
    import physics_refs
    for eps in STUDY_EPS:
        for beta in STUDY_BETA:
            assert abs(theory.theta_semianalytical(beta, eps) - physics_refs.theta_semianalytical(beta, eps)) < 1e-15
            assert theory.beta_limit(eps) == physics_refs.beta_limit(eps)
    cases = paper_study_cases()
    assert len(cases) == 35  # the pairs under the bound
    assert all(c["beta_p"] < physics_refs.beta_limit(c["eps"]) for c in cases)
