"""Pins of the oracle's iteration schedules, CPU only:

* ``pcg_block_jacobi``: its iterates, its iteration count and its stopping rule
  (unpreconditioned residual, ||r||_2 <= tol ||b||_2, x0 = 0, a cap on the products
  with S) against SciPy's conjugate gradients run with the same block-Jacobi
  preconditioner, built here from S's diagonal blocks with ``numpy.linalg.inv``;
* ``lm_iterate``, the Levenberg-Marquardt loop shared by every oracle solver, on
  models whose gain ratio is known in closed form: a linear least-squares problem
  (the quadratic model is exact, rho = 1), a scripted sequence of gain ratios, and
  steps that always raise the cost.  The expected damping values are the schedule of
  Madsen, Nielsen and Tingleff (2004, Sec. 3.2), worked out by hand below;
* the rejection of a step that lowers the cost by moving a point behind a camera.

Each pin is also run against the oracle with a planted mistake (a mutated copy of
the function, built here on the CPU) and must fail there: an off-by-one count, a stop
on the preconditioned residual, a wrong damping branch, a dropped clause of the
acceptance rule."""
import dataclasses
import inspect
import math
import textwrap

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import ba_oracle as O
from synth import make_arc_scene, make_config0, make_small_drive


def _mutant(fn, old, new):
    """A copy of oracle function ``fn`` with the source text ``old`` replaced by ``new``."""
    src = textwrap.dedent(inspect.getsource(fn))
    assert src.count(old) == 1, (fn.__name__, old)
    ns = dict(vars(O))
    exec(compile(src.replace(old, new), f"<mutant {fn.__name__}>", "exec"), ns)
    return ns[fn.__name__]


def _fails(check, *args):
    try:
        check(*args)
    except AssertionError:
        return True
    return False


# ----------------------------------------------------------------------------- PCG

def _system(scene, lam=1e-4):
    p = O.Problem.from_scene(scene)
    H, g, _, _, _ = O.normal_equations(p)
    D = O.damping_diag(H.diagonal())
    nf = int((~p.fixed).sum())
    S, b, _, _ = O.schur_blocks(H, g, D, lam, 6 * nf)
    return S, b


_SYSTEMS = {}


def _get_system(name):
    if name not in _SYSTEMS:
        _SYSTEMS[name] = _system(make_config0() if name == "config0" else make_small_drive(n_cams=12, n_pts=600, seed=5))
    return _SYSTEMS[name]


def _scipy_cg(S, b, tol, cap):
    """SciPy CG with M^-1 = blockdiag(inv(S_aa)), x0 = 0, rtol = tol, atol = 0."""
    nb = b.size // 6
    Minv = np.stack([np.linalg.inv(S[6 * a:6 * a + 6, 6 * a:6 * a + 6]) for a in range(nb)])
    M = spla.LinearOperator(S.shape, matvec=lambda r: np.einsum("aij,aj->ai", Minv, r.reshape(nb, 6)).ravel())
    xs = []
    x, info = spla.cg(S, b, x0=np.zeros_like(b), rtol=tol, atol=0.0, maxiter=cap, M=M,
                      callback=lambda xk: xs.append(np.array(xk)))
    return x, xs


def _check_pcg(pcg, S, b, tol, cap):
    """The oracle's PCG takes SciPy's iterates and stops where SciPy stops."""
    x_ref, xs = _scipy_cg(S, b, tol, cap)
    x, it = pcg(S, b, tol, cap)
    assert it == len(xs), (it, len(xs))
    assert np.linalg.norm(x - x_ref) <= 1e-6 * np.linalg.norm(x_ref)
    bn = np.linalg.norm(b)
    for k in range(1, it + 1):
        xk, ik = pcg(S, b, tol, k)
        assert ik == k
        assert np.linalg.norm(xk - xs[k - 1]) <= 1e-6 * np.linalg.norm(xs[k - 1]), k
        rel = np.linalg.norm(b - S @ xs[k - 1]) / bn
        if k < it:
            assert rel > tol * (1 - 1e-6), (k, rel)   # not yet converged below the count
    if it < cap:
        assert np.linalg.norm(b - S @ x) <= tol * bn * (1 + 1e-6)


@pytest.mark.parametrize("name", ["config0", "drive"])
@pytest.mark.parametrize("tol,cap", [(1e-6, 500), (1e-10, 500), (1e-10, 7)])
def test_pcg_iterates_and_count_match_scipy_cg(name, tol, cap):
    S, b = _get_system(name)
    _check_pcg(O.pcg_block_jacobi, S, b, tol, cap)
    if cap == 7:
        assert O.pcg_block_jacobi(S, b, tol, cap)[1] == 7   # a cap smaller than convergence


@pytest.mark.parametrize("old,new", [
    ("while it < max_iters:", "while it <= max_iters:"),                       # one product too many
    ("if math.sqrt(float(r @ r)) <= tol * bn:",                                # preconditioned residual
     "if math.sqrt(abs(float(r @ prec(r)))) <= tol * math.sqrt(abs(float(b @ prec(b)))):"),
    ("if math.sqrt(float(r @ r)) <= tol * bn:", "if math.sqrt(float(r @ r)) <= tol:"),  # absolute tol
    ("beta = rz_new / rz", "beta = rz_new / rz * 0.999"),
])
def test_pcg_pin_fails_on_a_planted_mistake(old, new):
    bad = _mutant(O.pcg_block_jacobi, old, new)
    assert any(_fails(_check_pcg, bad, *_get_system(name), tol, cap)
               for name in ("config0", "drive") for tol, cap in [(1e-3, 500), (1e-4, 500), (1e-6, 500), (1e-8, 500), (1e-10, 7)])


# ----------------------------------------------------------------------------- LM schedule

def _opts(n, lam0):
    return O.LMOptions(max_iters=n, lambda0=lam0)


def _run_linear(lm_iterate, n=8, lam0=1e3):
    """Linear least squares C(x) = |A x - y|^2 / 2: the quadratic model is exact, so
    every gain ratio is 1 and every step is accepted."""
    rng = np.random.default_rng(3)
    A = rng.normal(size=(40, 7)) * np.array([1, 3, 0.5, 10, 2, 1, 7])
    y = rng.normal(size=40)
    n_lin = [0]

    def cost_fn(x):
        e = A @ x - y
        return 0.5 * float(e @ e), 0

    def linearize(x):
        n_lin[0] += 1
        return A.T @ A, A.T @ (A @ x - y)

    def solve(x, H, g, D, lam):
        return np.linalg.solve(H + lam * np.diag(D), -g), 0

    _, out = lm_iterate(np.zeros(7), _opts(n, lam0), cost_fn, linearize, solve, lambda x, d: x + d)
    return out, n_lin[0]


def _check_linear(lm_iterate):
    out, n_lin = _run_linear(lm_iterate)
    assert all(out.accepted)
    assert np.allclose(out.rhos, 1.0, rtol=0, atol=1e-9)
    # rho = 1: lambda <- lambda * max(1/3, 1 - 1^3) = lambda / 3
    expect = [1e3 / 3 ** k for k in range(8)]
    assert np.allclose(out.lambdas, expect, rtol=1e-12, atol=0)
    assert out.nus == [2.0] * 8
    assert n_lin == 8                      # a fresh linearisation after every accept
    assert all(b < a for a, b in zip(out.iter_cost, out.iter_cost[1:]))


def test_lm_linear_least_squares_divides_lambda_by_three():
    _check_linear(O.lm_iterate)


# A one-unknown model with fixed H = 1 and g = 1 whose trial cost is scripted so the
# k-th gain ratio is RHOS[k]: the model's own predicted decrease of a step d is
# -g d - H d^2 / 2.
RHOS = [0.9, 0.5, 5e-4, -1.0, 2.0, 1.0, 0.25, 9e-4, 0.0011, 0.75]
# lambda used by each iteration, from lambda0 = 1e-2, nu = 2 (hand-worked):
#  it 1 rho 0.9   accept  factor max(1/3, 1 - 0.8^3)     = 0.488           nu 2
#  it 2 rho 0.5   accept  factor 1 - 0^3                 = 1               nu 2
#  it 3 rho 5e-4  reject  factor nu = 2                                     nu 4
#  it 4 rho -1    reject  factor 4                                          nu 8
#  it 5 rho 2     accept  factor max(1/3, 1 - 27)        = 1/3             nu 2
#  it 6 rho 1     accept  factor 1/3                                        nu 2
#  it 7 rho 0.25  accept  factor 1 - (-0.5)^3            = 1.125           nu 2
#  it 8 rho 9e-4  reject  factor 2                                          nu 4
#  it 9 rho .0011 accept  factor 1 - (-0.9978)^3         = 1.993414509352  nu 2
#  it 10 rho 0.75 accept  factor 1 - 0.5^3               = 0.875           nu 2
LAMS = [1e-2, 4.88e-3, 4.88e-3, 9.76e-3, 3.904e-2, 1.3013333333333333e-2, 4.337777777777778e-3,
        4.88e-3, 9.76e-3, 1.945572561127552e-2]
LAM_FINAL = 1.702375990986608e-2
NUS = [2.0, 2.0, 4.0, 8.0, 2.0, 2.0, 2.0, 4.0, 2.0, 2.0]
ACC = [True, True, False, False, True, True, True, False, True, True]


def _run_scripted(lm_iterate, rhos, lam0, C0=100.0):
    calls = {"trial": 0, "lin": 0}

    def cost_fn(st):
        return st["C"], st.get("masked", 0)

    def linearize(st):
        calls["lin"] += 1
        return np.array([[1.0]]), np.array([1.0])

    def solve(st, H, g, D, lam):
        return np.linalg.solve(H + lam * np.diag(D), -g), 0

    def apply(st, d):
        k = calls["trial"]
        calls["trial"] += 1
        dL = float(-1.0 * d[0] - 0.5 * d[0] * d[0])
        return {"C": st["C"] - rhos[k] * dL}

    _, out = lm_iterate({"C": C0}, _opts(len(rhos), lam0), cost_fn, linearize, solve, apply)
    return out, calls


def _check_scripted(lm_iterate):
    out, calls = _run_scripted(lm_iterate, RHOS, 1e-2)
    assert np.allclose(out.rhos, RHOS, rtol=1e-9, atol=1e-12)
    assert out.accepted == ACC
    assert np.allclose(out.lambdas, LAMS, rtol=1e-12, atol=0)
    assert out.nus == NUS
    assert calls["lin"] == 1 + sum(ACC[:-1])   # reused after a reject
    # the accepted-state cost after each iteration
    c, expect = 100.0, [100.0]
    for rho, lam, acc in zip(RHOS, LAMS, ACC):
        d = -1.0 / (1.0 + lam)
        if acc:
            c -= rho * (-d - 0.5 * d * d)
        expect.append(c)
    assert np.allclose(out.iter_cost, expect, rtol=1e-14)
    assert out.status == O.STATUS_OK
    # lambda after the last iteration: the next iteration's lambda
    out2, _ = _run_scripted(lm_iterate, RHOS + [0.5], 1e-2)
    assert out2.lambdas[-1] == pytest.approx(LAM_FINAL, rel=1e-12)


def test_lm_schedule_follows_scripted_gain_ratios():
    _check_scripted(O.lm_iterate)


def _check_clamps(lm_iterate):
    """Every step raises the cost: lambda_n = 1e-4 * 2^(n(n+1)/2), clamped at 1e16,
    which ends the run with STATUS_DAMPING; at the lower end lambda stays at 1e-12."""
    out, _ = _run_scripted(lm_iterate, [-1.0] * 14, 1e-4)
    assert not any(out.accepted)
    expect = [1e-4, 2e-4, 8e-4, 6.4e-3, 1.024e-1, 3.2768, 209.7152, 26843.5456, 6.8719476736e6,
              3.5184372088832e9, 3.6028797018963968e12, 7.378697629483821e15, 1e16, 1e16]
    assert np.allclose(out.lambdas, expect, rtol=1e-12, atol=0)
    assert out.nus == [2.0 ** (k + 2) for k in range(14)]
    assert out.status == O.STATUS_DAMPING
    assert out.iter_cost == [100.0] * 15
    low, _ = _run_scripted(lm_iterate, [1.0] * 6, 1e-11)   # rho = 1: lambda / 3, floored at 1e-12
    assert np.allclose(low.lambdas, [1e-11, 1e-11 / 3, 1e-11 / 9, 1e-12, 1e-12, 1e-12], rtol=1e-12, atol=0)
    assert low.status == O.STATUS_OK


def test_lm_all_rejected_steps_double_nu_and_clamp_at_the_upper_bound():
    _check_clamps(O.lm_iterate)


def test_lm_failed_solve_is_a_rejected_step():
    """A damped system that the solver reports as not positive definite (d = None)
    counts as a rejected step: lambda * nu, nu * 2, no trial cost."""
    def solve(st, H, g, D, lam):
        return (None, 0) if lam < 1e-3 else (np.linalg.solve(H + lam * np.diag(D), -g), 0)

    trials = []

    def apply(st, d):
        trials.append(d)
        return {"C": st["C"] - 0.5 * float(-d[0] - 0.5 * d[0] * d[0])}

    _, out = O.lm_iterate({"C": 10.0}, _opts(4, 2e-4), lambda st: (st["C"], 0),
                          lambda st: (np.array([[1.0]]), np.array([1.0])), solve, apply)
    assert out.accepted == [False, False, True, True]
    assert np.allclose(out.lambdas, [2e-4, 4e-4, 1.6e-3, 1.6e-3], rtol=1e-12)   # rho 0.5: factor 1
    assert math.isnan(out.rhos[0]) and math.isnan(out.rhos[1])
    assert len(trials) == 2


LM_MUTANTS = [
    ("lam = lam * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)",
     "lam = lam * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 2)"),            # wrong exponent
    ("lam = lam * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)",
     "lam = lam * min(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)"),            # min for max
    ("            nu = 2.0\n            lin = None", "            lin = None"),  # nu not reset on accept
    ("            nu = 2.0 * nu", "            nu = nu"),                       # nu not doubled
    ("            lam = lam * nu\n", "            lam = lam * 2.0\n"),            # fixed factor 2
    ("rho > ACCEPT_RHO", "rho > 0"),                                          # threshold
    ("dL = 0.5 * float(delta @ (lam * D * delta - g))",
     "dL = 0.5 * float(delta @ (-lam * D * delta - g))"),                    # damped model in dL
    ("lam = min(max(lam, LAMBDA_MIN), LAMBDA_MAX)", "lam = max(lam, LAMBDA_MIN)"),  # no upper clamp
    ("lam = min(max(lam, LAMBDA_MIN), LAMBDA_MAX)", "lam = min(lam, LAMBDA_MAX)"),  # no lower clamp
    ("            lin = None\n        else:", "        else:"),                   # stale linearisation
]


@pytest.mark.parametrize("old,new", LM_MUTANTS)
def test_lm_schedule_pins_fail_on_a_planted_mistake(old, new):
    bad = _mutant(O.lm_iterate, old, new)
    assert any(_fails(chk, bad) for chk in (_check_linear, _check_scripted, _check_clamps))


# ----------------------------------------------------------------------------- masked steps

def _masking_case():
    """A point whose observations are 60 px off in both coordinates, and a step that
    moves only that point behind every camera: the trial state masks its observations,
    so the cost falls by their whole contribution.  lambda0 is chosen so that the
    predicted decrease is positive and the gain ratio about 2e-3, above the threshold."""
    s = make_arc_scene(4, 40, seed=17, sigma=0.3)
    p = O.Problem.from_scene(s)
    j = 5
    sel = p.pt == j
    p.uv[sel] += 60.0
    nf = int((~p.fixed).sum())
    H, g = O.normal_equations(p)[:2]
    D = O.damping_diag(H.diagonal())
    delta = np.zeros(6 * nf + 3 * p.n_pts)
    sl = slice(6 * nf + 3 * j, 6 * nf + 3 * j + 3)
    delta[sl] = np.array([0.0, 0.0, -60.0]) - p.X[j]
    C, m0 = O.cost_and_masked(p)
    Cn, m1 = O.cost_and_masked(p, *O.apply_step(p, delta[:6 * nf], delta[6 * nf:]))
    drop = C - Cn
    a = float(delta[sl] @ (D[sl] * delta[sl]))
    c = float(g[sl] @ delta[sl])
    lam = max((c + 1000.0 * drop) / a, 1e-12)
    dL = 0.5 * float(delta @ (lam * D * delta - g))
    return p, delta, lam, (C, Cn, m0, m1, dL)


def _check_masked_step_rejected(lm_loop):
    p, delta, lam, (C, Cn, m0, m1, dL) = _masking_case()
    assert m1 > m0 and Cn < C and dL > 0 and (C - Cn) / dL > 1e-3   # the step would pass the gain test
    out = lm_loop(p, O.LMOptions(max_iters=1, lambda0=lam), lambda q, H, g, D, lm, o: (delta, 0))
    assert out.accepted == [False]
    assert out.iter_cost == [C, C]
    assert out.rhos[0] > 1e-3


def test_step_that_masks_observations_is_rejected_although_it_lowers_the_cost():
    _check_masked_step_rejected(O._lm_loop)


def test_masked_step_pin_fails_without_the_masking_clause():
    bad_iter = _mutant(O.lm_iterate, " and masked_n <= masked", "")
    ns = dict(vars(O))
    ns["lm_iterate"] = bad_iter
    src = textwrap.dedent(inspect.getsource(O._lm_loop))
    exec(compile(src, "<_lm_loop over mutant>", "exec"), ns)
    assert _fails(_check_masked_step_rejected, ns["_lm_loop"])
