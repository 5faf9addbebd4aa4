"""Write oracle eigenvalue references for the seeded systems (calls only oracle/ and gen/).

usage: python tests/golden/make_golden.py c1 [c2 p5 c3rows ...]
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


# sampled output rows of the 108^3 / Nocc = 432 system: the D, exchange and
# response terms separately, for the seeded two-trial block of gen.trials_random
C3_ROWS = [0, 215, 431]
C3_NB = 2


def c3_rows():
    import oracle.planewave as pw
    pw._WORKERS = len(os.sched_getaffinity(0))
    from gen import trials_random
    s = make_system(CONFIGS["c3"])
    a = trials_random(s, C3_NB)
    t0 = time.time()

    def say(msg):
        print(f"[c3rows] {msg} t={time.time() - t0:.0f}s", flush=True)

    d = oracle.apply_liouville(s, a, terms=oracle.TERM_D, rows=C3_ROWS, progress=say)
    k1d = oracle.apply_liouville(s, a, terms=oracle.TERM_K1D, rows=C3_ROWS, progress=say)
    k1e = oracle.apply_liouville(s, a, terms=oracle.TERM_K1E, rows=C3_ROWS, progress=say)
    path = os.path.join(HERE, "rows_c3.npz")
    np.savez(path, rows=np.asarray(C3_ROWS), nb=C3_NB, d=d, k1d=k1d, k1e=k1e,
             source=np.asarray("oracle.apply_liouville(terms=D, K1D, K1E separately, rows) on "
                               "gen.trials_random(gen.make_system(CONFIGS['c3']), 2)"))
    say(f"wrote {path}")


def main(names):
    for name in names:
        if name == "c3rows":
            c3_rows()
            continue
        cfg = CONFIGS[name]
        s = make_system(cfg)
        tol = 1e-8 if name in ("c1", "p5") else 1e-7
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
