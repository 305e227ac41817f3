"""The oracle's aggregation, mean-based coarse solve, Newton mean stiffness
and Adam step against hand-worked cases and closed forms (tests/oracle_pins.py
states each)."""
import numpy as np

from oracle import amg, coarse, fem, nn
from oracle import newton as onl

import oracle_pins as pins


def test_aggregation_hand_worked_passes():
    assert pins.pin_aggregate(amg.aggregate)


def test_aggregation_hand_graph_strength_pattern():
    """The hand graph's strong couplings are the ones its docstring lists."""
    S, _ = pins.hand_graph()
    d = np.abs(np.diag(S))
    strong = {(s, t) for s in range(6) for t in range(6)
              if s < t and S[s, t] != 0 and abs(S[s, t]) >= 0.08 * np.sqrt(d[s] * d[t])}
    assert strong == {(0, 2), (1, 3), (2, 4), (3, 4), (4, 5), (3, 5)}


def test_mean_exact_coarse_is_dense_kronecker_solve():
    C, G, af, Cd = pins.coarse_fixture()
    assert pins.pin_mean_exact_coarse(coarse.MeanExactCoarse, C, G, af, Cd)


def test_newton_mean_stiffness_closed_form():
    for a1, a2 in [(0.0, 0.5), (1.0, 0.0), (0.3, 0.5)]:
        nl, ijk, val = pins.newton_fixture(a1, a2)
        assert pins.pin_mean_stiffness(onl.NLProblem.mean_stiffness, nl, ijk, val,
                                       fem.assemble), (a1, a2)


def test_newton_mean_stiffness_at_zero_is_mean_stiffness_of_linear_problem():
    nl, _, _ = pins.newton_fixture()
    K0 = fem.assemble(nl.xy, nl.tri, nl.dof, nl.n, nl.coef[:1])[0].toarray()
    got = nl.mean_stiffness(np.zeros((nl.n, nl.P))).toarray()
    assert np.allclose(got, K0, rtol=1e-13, atol=1e-14 * np.abs(K0).max())


def test_adam_hand_worked_trajectories():
    assert pins.pin_adam(nn.adam_step)
