"""Write plan_breakpoints.json from the oracle's plan rule (calls only oracle/).

For each accuracy and each scheme bound theta_level, and s = 0..12, records
the oracle's (level, s, products) at theta_level * 2^s and at the next float
above it. Run from the repository root:  python tests/golden/make_plan_breakpoints.py
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import plan as P  # noqa: E402


def main():
    out = {"source": "oracle/plan.py rule over Tables 1-2 bounds (min of cosine and sine bound per scheme)",
           "cases": []}
    for acc in ("double", "single"):
        for level, th in P.THETA[acc].items():
            for s in range(0, 13):
                x = math.ldexp(th, s)
                for t in (x, math.nextafter(x, math.inf), math.nextafter(x, 0.0)):
                    lv, ss, pr = P.plan(t, acc)
                    out["cases"].append({"accuracy": acc, "norm1": t.hex(), "level": lv, "s": ss,
                                         "products": pr})
        for t in (0.0, 5e-324, 1e-300, 1e-8, 1.0, 2.0, 16.0, 64.0, 1024.0, 1e8, 1e300):
            lv, ss, pr = P.plan(t, acc)
            out["cases"].append({"accuracy": acc, "norm1": t.hex(), "level": lv, "s": ss, "products": pr})
    with open(os.path.join(HERE, "plan_breakpoints.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
