"""Write tests/golden/reference_values.json: optimal values F* of the seeded
workloads, computed only with oracle/ (the textbook interior-point solver in
oracle/ipm.py, which shares nothing with the dual first-order method).

    python tests/golden/make_reference_values.py [--large]

The large instance (n=8192, p=4096) takes minutes of CPU time.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle.ipm import ipm_qp  # noqa: E402
from paper_1504_05708_amd import gen  # noqa: E402

OUT = os.path.join(HERE, "reference_values.json")


def fstar(qp):
    t = time.time()
    x, f, z = ipm_qp(qp.Q, qp.q, qp.G, qp.g, qp.lb, qp.ub, tol=1e-10)
    kkt = float(np.max(np.abs(x - np.clip(x - (qp.Q @ x + qp.q + qp.G.T @ z), qp.lb, qp.ub))))
    feas = float(np.linalg.norm(np.maximum(qp.G @ x + qp.g, 0)))
    return dict(fstar=f, kkt_residual=kkt, feas=feas, lam_norm=float(np.linalg.norm(z)),
                seconds=round(time.time() - t, 1))


def main():
    vals = json.load(open(OUT)) if os.path.exists(OUT) else {}
    vals["config0"] = dict(fstar(gen.config0()), recipe="random_dense_qp(50, 25, seed=0, reg=0.1)")
    if "--large" in sys.argv:
        qp = gen.config1()
        vals["config1_f64"] = dict(fstar(qp), recipe="random_dense_qp(8192, 4096, seed=1, reg=0.01)")
        print("config1_f64", vals["config1_f64"], flush=True)
        vals["config1_f32"] = dict(fstar(qp.rounded(np.float32)),
                                   recipe="config1 with Q, G rounded to float32 (RNE)")
        print("config1_f32", vals["config1_f32"], flush=True)
    json.dump(vals, open(OUT, "w"), indent=1, sort_keys=True)
    print(json.dumps(vals, indent=1))


if __name__ == "__main__":
    main()
