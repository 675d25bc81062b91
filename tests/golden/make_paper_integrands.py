"""Writes paper_integrands_d3.json: the Sec. 4 test functions f1..f7 of
arXiv 2511.01573 at d = 3 on [0,1]^3, as parameters of the seeded families
plus their exact integrals from the closed forms in tests/closed_forms.py.

The paper prints the seven formulas (Sec. 4, the list of integrands) but no
integral values; the values here are the analytic integrals of those formulas.
f6 uses the reading "zero when x_i > (3+i)/10 for ANY i".
Run from the repository root: python tests/golden/make_paper_integrands.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
import closed_forms as cf  # noqa: E402

out = {"citation": "arXiv 2511.01573, Sec. 4 (test integrands f1..f7; stopping rule)",
       "domain": "[0,1]^3", "d": 3, "cases": []}
for k in range(1, 8):
    fam, a, u = cf.paper_params(k, 3)
    out["cases"].append({"name": f"f{k}", "family": fam, "a": a, "u": u,
                         "exact": str(cf.exact(fam, a, u))})
with open(os.path.join(HERE, "paper_integrands_d3.json"), "w") as fh:
    json.dump(out, fh, indent=1)
    fh.write("\n")
