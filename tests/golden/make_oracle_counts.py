"""Write tests/golden/oracle_outer_counts.json: the oracle's outer iteration
counts to tol for the named workloads (exact subdomain solves, Jacobi
Robin-Schwarz, global residual checked after every outer iteration).

Calls only the oracle and the seeded input generators. Usage:
    python tests/golden/make_oracle_counts.py c1 c2
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import assemble as A  # noqa: E402
from oracle import mesh as M  # noqa: E402
from oracle import partition as P  # noqa: E402
from oracle import schwarz as S  # noqa: E402
from oracle import subdomain as SD  # noqa: E402
from synth import workload  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_outer_counts.json")


def count(name, seed=0, block=25):
    wl = workload(name, seed=seed)
    m = M.BoxMesh(wl.ne, wl.lengths, wl.bc)
    part = P.BoxPartition(m, wl.cuts)
    drho = wl.drho()
    f = A.load_from_density(m, drho, wl.G)
    fs = [SD.density_load(part, s, drho, wl.G) for s in part.subs]
    orc = S.SchwarzOracle(part, wl.p, "fdm")
    lam = orc.zero_data()
    n = 0
    t0 = time.time()
    while True:
        saved, n0 = lam, n
        for _ in range(block):
            u = orc.subdomain_solves(fs, lam)
            lam = orc.exchange(u, lam)
            n += 1
        res = A.residual_norm(m, orc.glue(u), f)
        print(name, n, res, round(time.time() - t0, 1), flush=True)
        if res <= wl.tol:
            break
    lam, n = saved, n0  # replay the last block one iteration at a time
    while True:
        u = orc.subdomain_solves(fs, lam)
        lam = orc.exchange(u, lam)
        n += 1
        res = A.residual_norm(m, orc.glue(u), f)
        if res <= wl.tol:
            return {"workload": name, "seed": seed, "tol": wl.tol, "p": wl.p, "outer_iters": n,
                    "rel_residual": res}


if __name__ == "__main__":
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in sys.argv[1:]:
        r = count(name)
        data[f"{name}_seed{r['seed']}"] = r
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
        print(r, flush=True)
