"""Writes e1_errors.json: the oracle's total L2 error on the paper's
manufactured-solution problem (Sec. 5.1) at the sizes of Table tab:cpu that a
CPU direct solve finishes (p=1 on 16^3 and p=3 on 8^3; 65,536 DOFs each).
Calls only the oracle.  Run from the repository root:
    python tests/golden/make_e1.py
"""
import json
import os
import sys
import time

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))

from oracle import solve  # noqa: E402
from oracle.dg import DG  # noqa: E402
from oracle.problem import Problem  # noqa: E402
from workload import get_config  # noqa: E402

out = []
for p, n in ((1, 16), (3, 8), (1, 8), (3, 4)):
    cfg = get_config("e1").with_(n=(n, n, n), p=p)
    dg = DG(Problem(cfg))
    t = time.time()
    x, hist = solve.newton(dg, tol=1e-12)
    errs = solve.l2_errors(dg, x)
    out.append(dict(p=p, n=n, dofs=dg.N, err_phi=errs[0], err_c1=errs[1], total=errs[0] + errs[1],
                    newton_residuals=[float(h) for h in hist], seconds=time.time() - t))
    print(out[-1], flush=True)
with open(os.path.join(os.path.dirname(__file__), "e1_errors.json"), "w") as f:
    json.dump(dict(generator="tests/golden/make_e1.py", results=out), f, indent=1)
