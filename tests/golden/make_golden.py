"""Write oracle reference values for the larger parity cases.

Calls only the oracle.  Usage:  python tests/golden/make_golden.py NAME [NAME ...]
Each NAME selects one case below; the result goes to tests/golden/NAME.json
with, after every step, log Z/V and the gauge-invariant spectra of the step:

* ``resplit_s``  singular values of T^(k) / c_k at the step's re-split;
* ``bond_sig``   the kept bond-swap singular values and ``bond_kept``;
* ``sq_s``       for each transverse position, the squeezer singular values
                 (relative to the largest, first D + 1) and ``sq_kept``
                 (null for an identity squeezer);
* ``triad_kept`` kept columns of the four triad isometries (null: identity);
* ``gu_wen_x``   the Gu-Wen ratio X with the open leg along each axis.

A GPU run of the same flow is compared with these step by step.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import trg  # noqa: E402

BASE = 0x2507219090000000

CASES = {
    # triad-ATRG, beta 0.1497, h 0, L = 2^10 per axis (40 steps), D 16, r 7,
    # sketch width 2D, one power iteration
    "triad_d16_l1024": dict(beta=0.1497, h=0.0, D=16, nsteps=40, seed=BASE + 2000, method="triad"),
    # the same at D 32 for the first 12 steps (L = 8 per axis)
    "triad_d32_12steps": dict(beta=0.1497, h=0.0, D=32, nsteps=12, seed=BASE + 3000, method="triad"),
    # a field case at D 16, 16 steps
    "triad_d16_h1e-4_16steps": dict(beta=0.1497, h=1e-4, D=16, nsteps=16, seed=BASE + 3001, method="triad"),
    # a field case at D 32, 12 steps
    "triad_d32_h1e-4_12steps": dict(beta=0.1497, h=1e-4, D=32, nsteps=12, seed=BASE + 3001, method="triad"),
}

# The mixed-precision grid at D 16: beta in {0.1497, 0.140, 0.160} x h in {0, 1e-4},
# L = 2^20 per axis (80 steps); run i draws its sketches with seed BASE + 3000 + i.
# "_t7" variants use the multiplet tolerance 1e-7 that the mixed-precision
# comparisons run at (the FP64 cases use the default 1e-9).
_GRID = [(0.1497, 0.0), (0.1497, 1e-4), (0.140, 0.0), (0.140, 1e-4), (0.160, 0.0), (0.160, 1e-4)]
for _i, (_b, _h) in enumerate(_GRID):
    _name = "grid_d16_b%.4f_h%g" % (_b, _h)
    CASES[_name] = dict(beta=_b, h=_h, D=16, nsteps=80, seed=BASE + 3000 + _i, method="triad")
    CASES[_name + "_t7"] = dict(beta=_b, h=_h, D=16, nsteps=80, seed=BASE + 3000 + _i, method="triad",
                                tau_deg=1e-7)

# ILO triad-ATRG (Sec. II C): the bond swap keeps r_bond D values, sketch
# width (r_bond + 1) D; the paper's own runs use r_bond = 5
CASES["ilo_d16_rb2_16steps"] = dict(beta=0.1497, h=0.0, D=16, nsteps=16, seed=BASE + 4000, method="triad",
                                    r_bond=2, sketch_mult=3)
CASES["ilo_d12_rb6_8steps"] = dict(beta=0.1497, h=1e-4, D=12, nsteps=8, seed=BASE + 4001, method="triad",
                                   r_bond=6, sketch_mult=7)
CASES["ilo_d16_rb5_6steps"] = dict(beta=0.1497, h=0.0, D=16, nsteps=6, seed=BASE + 4002, method="triad",
                                   r_bond=5, sketch_mult=6)

# Multiplet-tolerance study: the D 16 flow of triad_d16_l1024 at other tolerances
# (0: only exact ties are kept together, i.e. the plain cap at D).
for _t in (0.0, 1e-12, 1e-7):
    CASES["tau_d16_l1024_t%g" % _t] = dict(beta=0.1497, h=0.0, D=16, nsteps=40, seed=BASE + 2000,
                                           method="triad", tau_deg=_t)


def _spectra(rec, D):
    out = {}
    out["resplit_s"] = [float(v) for v in rec["s"]]
    b = rec["bond"]
    out["bond_kept"] = int(b["kept"])
    out["bond_sig"] = [float(v) for v in b["sig"][: b["kept"]]]
    sq_s, sq_k = [], []
    for pos in range(3):
        q = rec.get("sq%d" % pos, {})
        if q.get("identity", False) or "kept" not in q:
            sq_s.append(None)
            sq_k.append(None)
        else:
            sq_s.append([float(v) for v in q["s"][: D + 1]])
            sq_k.append(int(q["kept"]))
    out["sq_s"] = sq_s
    out["sq_kept"] = sq_k
    tk = []
    for nm in ("UA", "UX", "UY", "UD"):
        q = rec.get(nm, {})
        tk.append(None if q.get("identity", False) or "kept" not in q else int(q["kept"]))
    out["triad_kept"] = tk
    return out


def main(name):
    c = CASES[name]
    prm = trg.Params(D=c["D"], seed=c["seed"], tau_deg=c.get("tau_deg", 1e-9), r_bond=c.get("r_bond", 1),
                     sketch_mult=c.get("sketch_mult", 2))
    st = trg.init_ising(c["beta"], c["h"], 4)
    out = dict(case=name, params=c, log_z=[], seconds=[], spectra=[], gu_wen_x=[])
    for i in range(c["nsteps"]):
        t0 = time.time()
        trg.rg_step(st, i % 4, prm, c["method"])
        out["log_z"].append(trg.log_z_per_site(st))
        out["seconds"].append(time.time() - t0)
        out["spectra"].append(_spectra(st.log[-1], c["D"]))
        out["gu_wen_x"].append([trg.gu_wen_x(st, ax) for ax in range(4)])
        gaps = [v.get("gap") for v in st.log[-1].values() if isinstance(v, dict) and v.get("gap") is not None]
        print("%s step %d log_z %.16f  %.1fs  min gap %s" % (name, i, out["log_z"][-1], out["seconds"][-1],
                                                            min(gaps) if gaps else None), flush=True)
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        main(nm)
