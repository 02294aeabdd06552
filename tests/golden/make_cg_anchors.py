"""Writes cg_anchors.json: iteration counts of the oracle's solvers at the
full workload sizes, used as anchors (+-1) by the GPU tests.  Calls only
`oracle` and `inputs` (run: python tests/golden/make_cg_anchors.py)."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import inputs  # noqa: E402
import oracle  # noqa: E402


def main():
    out = {}
    for name, gen, n in (("hpcg27_104", inputs.hpcg27, 104), ("hpcg27_128", inputs.hpcg27, 128),
                         ("aniso7_128", inputs.aniso7, 128)):
        p = gen(n)
        x, it, rel, st = oracle.cg(p.row_ptr, p.col, p.val, p.b, tol=1e-10)
        out[f"cg_{name}_tol1e-10"] = {"iters": it, "status": st, "relres": rel}
        print(name, it, st, rel, flush=True)
    L = inputs.hpcg27_levels(104, 4)
    lv = [{"row_ptr": l["problem"].row_ptr, "col": l["problem"].col, "val": l["problem"].val,
           "order": np.argsort(l["colour"], kind="stable").astype(np.int32), **({"f2c": l["f2c"]} if "f2c" in l else {})}
          for l in L]
    x, it, rel, st = oracle.pcg_mg(lv, L[0]["problem"].b, tol=1e-10)
    out["pcg_mg_hpcg27_104_4levels_tol1e-10"] = {"iters": it, "status": st, "relres": rel}
    print("pcg_mg 104", it, st, rel, flush=True)
    with open(os.path.join(HERE, "cg_anchors.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
