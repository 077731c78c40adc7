"""The oracle's pins catch plausible mistakes: each case below plants one
mistake in the oracle's source (a dropped term, a wrong sign, factor, index
or log base), loads the mutated module in place of oracle.dfom in a fresh
process, and runs the pin tests; at least one pin must fail (a pin that
runs past 30 s, as one whose method diverges does, counts as failed).  The
mistakes are planted on the CPU, in the oracle only."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle", "dfom.py")

# (name, exact source text, its mutated replacement)
MUTATIONS = [
    ("outer step 1/L_d instead of 1/(2 L_d)",
     "alpha = 0.0 if Ld == 0.0 else 1.0 / (2.0 * Ld)", "alpha = 0.0 if Ld == 0.0 else 1.0 / Ld"),
    ("L_d without the rho term",
     "denom = lam_min + rho * G_norm2", "denom = lam_min + 0.0 * rho * G_norm2"),
    ("k_in with log10",
     "math.sqrt(L_in / sigma_in) * math.log(arg)", "math.sqrt(L_in / sigma_in) * math.log10(arg)"),
    ("k_in without the square root",
     "math.ceil(math.sqrt(L_in / sigma_in) * math.log(arg))", "math.ceil((L_in / sigma_in) ** 0.25 * math.log(arg))"),
    ("FGM_sigma momentum with a sign error",
     "beta_in = (sqL - sqs) / (sqL + sqs)", "beta_in = (sqL + sqs) / (sqL + sqs) * 0.999"),
    ("pi^2/sigma certificate missing its factor 2",
     "float(pi @ pi) / (2.0 * sigma))", "float(pi @ pi) / (8.0 * sigma))"),
    ("gradient-mapping certificate with the wrong L term",
     "- gg / (2.0 * L)", "- gg / (0.5 * L)"),
    ("FW gap with only the lower side",
     "fw = float(np.sum(np.maximum(grad * (x - lb), grad * (x - ub))))",
     "fw = float(np.sum(grad * (x - lb)))"),
    ("dual gradient without g",
     "return G @ u + g - slack(G, g, u, lam, rho, eq)", "return G @ u - slack(G, g, u, lam, rho, eq)"),
    ("Lagrangian without the multiplier term",
     "return objective(Q, q, u) + float(lam @ r)", "return objective(Q, q, u) + 0.5 * float(lam @ r)"),
    ("augmented Lagrangian with rho instead of rho/2",
     "0.5 * rho * d * d - float(lam @ lam) / (2.0 * rho)", "rho * d * d - float(lam @ lam) / (2.0 * rho)"),
    ("inner gradient with G^T mu transposed sign",
     "return Q @ u + q + G.T @ mu", "return Q @ u + q - G.T @ mu"),
    ("augmented inner gradient without the projection",
     "w = np.where(_ineq(G, eq), np.maximum(v, 0.0), v)", "w = v"),
    ("projection onto K on the wrong side",
     "np.minimum(v, 0.0), 0.0)", "np.maximum(v, 0.0), 0.0)"),
    ("theta rule with 2 theta^2",
     "theta_next = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * theta * theta))",
     "theta_next = 0.5 * (1.0 + math.sqrt(1.0 + 2.0 * theta * theta))"),
    ("dual momentum over theta_k instead of theta_{k+1}",
     "beta = (theta - 1.0) / theta_next", "beta = (theta - 1.0) / (theta + 1.0)"),
    ("average with unit weights",
     "u_sum = u_sum + theta * u", "u_sum = u_sum + u"),
    ("FGM inner momentum over theta_k instead of theta_{k+1}",
     "yield (th - 1.0) / th_next", "yield (th - 1.0) / th"),
    ("inner step 2/L",
     "x = np.clip(y - grad(y) / L, lb, ub)        # x^{t+1}", "x = np.clip(y - 2.0 * grad(y) / L, lb, ub)"),
    ("lower rows of the user form with the wrong offset sign",
     "rows.append(-G[i]); off.append(lo - g[i])", "rows.append(-G[i]); off.append(g[i] - lo)"),
    ("outer test on G x instead of G x + g",
     "feas = dist_K(G @ x + g, eq)", "feas = dist_K(G @ x, eq)"),
]

CHILD = r'''
import sys, types
root, old, new = sys.argv[1], sys.argv[2], sys.argv[3]
sys.path.insert(0, root)
src = open(root + "/oracle/dfom.py").read()
assert src.count(old) >= 1, "mutation text not found"
src = src.replace(old, new)
import oracle
mod = types.ModuleType("oracle.dfom")
mod.__file__ = root + "/oracle/dfom.py"
sys.modules["oracle.dfom"] = mod
exec(compile(src, mod.__file__, "exec"), mod.__dict__)
oracle.dfom = mod
import pytest
sys.exit(pytest.main([root + "/tests/test_oracle_pins.py", "-x", "-q", "-p", "no:cacheprovider",
                      "-p", "no:randomly", "--timeout", "30", "--timeout-method", "thread"]))
'''


def _run(case):
    name, old, new = case
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, old, new], capture_output=True, text=True,
                       timeout=900, cwd=ROOT, env=env)
    return name, r.returncode, r.stdout[-2000:] + r.stderr[-2000:]


def test_mutation_texts_are_in_the_oracle():
    src = open(ORACLE).read()
    for name, old, _ in MUTATIONS:
        assert old in src, name


def test_every_planted_mistake_fails_a_pin():
    assert len(MUTATIONS) >= 20
    with ThreadPoolExecutor(max_workers=8) as ex:
        results = list(ex.map(_run, MUTATIONS))
    survived = [(name, out) for name, rc, out in results if rc == 0]
    broken = [(name, out) for name, rc, out in results if rc not in (0, 1)]
    assert not broken, broken[:2]
    assert not survived, [name for name, _ in survived]
