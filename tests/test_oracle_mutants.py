"""Planted mistakes: each pin of tests/oracle_pins.py must reject a copy of
the oracle function with one plausible mistake in it (a dropped term, a
wrong index or tie-break, a lost piece of state).  The copies are made from
the oracle's source text on the CPU and never leave this test."""
import inspect
import textwrap

import pytest

from oracle import amg, coarse, fem, geometric, nn
from oracle import newton as onl

import oracle_pins as pins


def _mutant(obj, old, new):
    """Recompile `obj` (function or class) with `old` replaced by `new` in
    its source, in a copy of its module's namespace."""
    src = textwrap.dedent(inspect.getsource(obj))
    assert src.count(old) >= 1, f"mutation site not found: {old!r}"
    ns = dict(inspect.getmodule(obj).__dict__)
    exec(compile(src.replace(old, new), f"<mutant of {obj.__qualname__}>", "exec"), ns)
    return ns[obj.__name__]


AGG_MUTANTS = [
    ("no pass-2 snapshot", "if snap[j] >= 0 and", "if agg[j] >= 0 and"),
    ("tie to the higher index", "abs(S[i, j]) > best_v", "abs(S[i, j]) >= best_v"),
    ("strength without square root", "np.sqrt(diag[i] * diag[j])", "(diag[i] * diag[j])"),
    ("strength against the smaller diagonal", "np.sqrt(diag[i] * diag[j])",
     "min(diag[i], diag[j])"),
    ("pass 1 ignores the neighbourhood", "if all(agg[j] < 0 for j in nbrs[i]):", "if True:"),
    ("pass 2 skipped", "    snap = agg.copy()\n", "    snap = agg.copy()\n    nbrs_saved = nbrs\n    nbrs = [[] for _ in nbrs]\n"),
]


@pytest.mark.parametrize("name,old,new", AGG_MUTANTS, ids=[m[0] for m in AGG_MUTANTS])
def test_aggregation_pin_rejects(name, old, new):
    assert pins.pin_aggregate(amg.aggregate)
    assert not pins.pin_aggregate(_mutant(amg.aggregate, old, new)), name


COARSE_MUTANTS = [
    ("G_0 scaling dropped", "/ self.alpha_fact[None, :]", ""),
    ("G_0 scaling inverted", "/ self.alpha_fact[None, :]", "* self.alpha_fact[None, :]"),
    ("G_0 as the squared norms", "/ self.alpha_fact[None, :]",
     "/ self.alpha_fact[None, :] ** 2"),
    ("wrong input term", "C[0].toarray()", "(C[0] + C[1]).toarray()"),
]


@pytest.mark.parametrize("name,old,new", COARSE_MUTANTS, ids=[m[0] for m in COARSE_MUTANTS])
def test_mean_exact_coarse_pin_rejects(name, old, new):
    C, G, af, Cd = pins.coarse_fixture()
    assert pins.pin_mean_exact_coarse(coarse.MeanExactCoarse, C, G, af, Cd)
    bad = _mutant(coarse.MeanExactCoarse, old, new)
    assert not pins.pin_mean_exact_coarse(bad, C, G, af, Cd), name


MS_MUTANTS = [
    ("vertex value instead of centroid", "ub.mean(axis=1)", "ub[:, 0]"),
    ("derivative of kappa", "self.kappa(ub.mean(axis=1))", "self.dkappa(ub.mean(axis=1))"),
    ("quadrature weights dropped", "(self.wq[None, :] * c *", "(c *"),
    ("input terms off by one", "self.psi[:, :self.L].T", "self.psi[:, 1:self.L + 1].T"),
]


@pytest.mark.parametrize("name,old,new", MS_MUTANTS, ids=[m[0] for m in MS_MUTANTS])
def test_mean_stiffness_pin_rejects(name, old, new):
    nl, ijk, val = pins.newton_fixture()
    assert pins.pin_mean_stiffness(onl.NLProblem.mean_stiffness, nl, ijk, val, fem.assemble)
    bad = _mutant(onl.NLProblem.mean_stiffness, old, new)
    assert not pins.pin_mean_stiffness(bad, nl, ijk, val, fem.assemble), name


ADAM_MUTANTS = [
    ("state not carried (t reset)", 'state["t"] += 1', 'state["t"] = 1'),
    ("no bias correction of m", "mh = m / (1.0 - beta1 ** t)", "mh = m"),
    ("no bias correction of v", "vh = v / (1.0 - beta2 ** t)", "vh = v"),
    ("moments swapped", "m = beta1 * state", "m = beta2 * state"),
    ("first moment not stored", "ms[j] = m;", "ms[j] = g;"),
]


@pytest.mark.parametrize("name,old,new", ADAM_MUTANTS, ids=[m[0] for m in ADAM_MUTANTS])
def test_adam_pin_rejects(name, old, new):
    assert pins.pin_adam(nn.adam_step)
    assert not pins.pin_adam(_mutant(nn.adam_step, old, new)), name


PROLONG_MUTANTS = [
    ("triangles swapped", "if a >= b:", "if a <= b:"),
    ("lower-triangle weight", "add(row, ci + 1, cj, a - b)", "add(row, ci + 1, cj, b - a)"),
    ("upper-triangle corner", "add(row, ci, cj + 1, b - a)", "add(row, ci + 1, cj, b - a)"),
    ("local coordinate", "a, b = (i % r) / r, (j % r) / r", "a, b = (j % r) / r, (i % r) / r"),
]


@pytest.mark.parametrize("name,old,new", PROLONG_MUTANTS, ids=[m[0] for m in PROLONG_MUTANTS])
def test_prolongation_pin_rejects(name, old, new):
    assert pins.pin_prolongation(geometric.prolongation)
    assert not pins.pin_prolongation(_mutant(geometric.prolongation, old, new)), name
