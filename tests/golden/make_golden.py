"""Write tests/golden/oracle_values.json from the oracle only.

Run from the repository root:  python tests/golden/make_golden.py
The stored numbers are regression anchors for the oracle itself (a later change
to its arithmetic must reproduce them or name the passage that justifies the
change); they are not pins of the method.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import dense, fastcheck  # noqa: E402
from paper_2405_19246_amd import inputs  # noqa: E402


def main():
    out = {"l3_n64_eps0.1_500_sweeps": [], "l4_n1000_eps0.01_fastcheck_200_sweeps": []}
    for s in (0, 1):
        u, h, eps = inputs.workload("l3_n64_eps0.1", instance=s)
        r = dense.sinkhorn(u, h, eps, itmax=500, check_every=500)
        out["l3_n64_eps0.1_500_sweeps"].append(
            dict(instance=s, W=r["W"], res=r["res"], log_phi_0_first=list(r["log_phi"][0, :4])))
    u, h, eps = inputs.workload("l4_n1000_eps0.01", instance=0)
    r = fastcheck.sinkhorn(u, h, eps, itmax=200, check_every=200)
    out["l4_n1000_eps0.01_fastcheck_200_sweeps"].append(
        dict(instance=0, W=r["W"], res=r["res"], log_phi_0_first=list(r["log_phi"][0, :4])))
    path = os.path.join(ROOT, "tests", "golden", "oracle_values.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
