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
