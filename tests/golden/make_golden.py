"""Write oracle eigenvalue references for the seeded systems (calls only oracle/ and gen/).

usage: python tests/golden/make_golden.py c1 [c2 ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from gen import CONFIGS, make_system  # noqa: E402


def main(names):
    for name in names:
        cfg = CONFIGS[name]
        s = make_system(cfg)
        tol = 1e-8 if name == "c1" else 1e-7
        t0 = time.time()
        calls = [0]

        def log_apply(X, _f=oracle.apply_transition):
            calls[0] += 1
            print(f"[{name}] apply #{calls[0]} nb={X.shape[0]} t={time.time() - t0:.0f}s", flush=True)
            return _f(s, X)

        diag = oracle.transition_diagonal(s)
        nocc, nc = diag.shape

        def matvec(V):
            return log_apply(V.T.reshape(-1, nocc, nc)).reshape(V.shape[1], -1).T

        th, X, rn, it, ok = oracle.davidson(matvec, diag, cfg.nroots, cfg.nb, tol=tol,
                                            max_iter=200)
        out = dict(config=name, nroots=cfg.nroots, nb=cfg.nb, tol=tol, converged=bool(ok),
                   iterations=int(it), roots_hartree=[float(x) for x in th],
                   residual_norms=[float(x) for x in rn], seconds=time.time() - t0,
                   source="oracle.davidson on gen.make_system(CONFIGS[%r])" % name)
        with open(os.path.join(HERE, f"roots_{name}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1"])
