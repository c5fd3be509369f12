"""Write oracle reference values of log Z/V for the larger parity cases.

Calls only the oracle.  Usage:  python tests/golden/make_golden.py NAME
NAME selects one case below; the result goes to tests/golden/NAME.json with
log Z/V after every step, so a GPU run can be compared step by step.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import trg  # noqa: E402

CASES = {
    # triad-ATRG, beta 0.1497, h 0, L = 2^10 per axis (40 steps), D 16, r 7,
    # sketch width 2D, one power iteration
    "triad_d16_l1024": dict(beta=0.1497, h=0.0, D=16, nsteps=40, seed=0x2507219090000000 + 2000, method="triad"),
    # the same at D 32 for the first 12 steps (L = 8 per axis)
    "triad_d32_12steps": dict(beta=0.1497, h=0.0, D=32, nsteps=12, seed=0x2507219090000000 + 3000, method="triad"),
    # a field case at D 16, 16 steps
    "triad_d16_h1e-4_16steps": dict(beta=0.1497, h=1e-4, D=16, nsteps=16, seed=0x2507219090000000 + 3001,
                                    method="triad"),
}


def main(name):
    c = CASES[name]
    prm = trg.Params(D=c["D"], seed=c["seed"])
    st = trg.init_ising(c["beta"], c["h"], 4)
    out = dict(case=name, params=c, log_z=[], seconds=[])
    for i in range(c["nsteps"]):
        t0 = time.time()
        trg.rg_step(st, i % 4, prm, c["method"])
        out["log_z"].append(trg.log_z_per_site(st))
        out["seconds"].append(time.time() - t0)
        gaps = [v.get("gap") for v in st.log[-1].values() if isinstance(v, dict) and v.get("gap") is not None]
        print("%s step %d log_z %.16f  %.1fs  min gap %s" % (name, i, out["log_z"][-1], out["seconds"][-1],
                                                            min(gaps) if gaps else None), flush=True)
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1])
