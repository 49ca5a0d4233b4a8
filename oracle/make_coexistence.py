"""Write ``lbm_inputs/coexistence.json``: Maxwell coexistence densities of the
Carnahan-Starling EOS (b = 4, R = 1; the values do not depend on a) on a grid
of reduced temperatures, and of the exponential pseudopotential with
psi0 = rho0 = 1, G = -10/3.  Calls only the oracle.  Run from the repo root:
    python oracle/make_coexistence.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import eos, ref  # noqa: E402


def main():
    table = []
    for i in range(0, 91):
        t = round(0.50 + 0.005 * i, 4)
        p = ref.make_params(dict(nx=1, ny=1, nz=1, G=-1.0, eos_a=0.5, T_over_Tc=t,
                                 s_e=1.0, s_nu=1.0, s_q=1.0, s_pi=1.0))
        rl, rv = eos.maxwell(ref.pressure_fn(p), 1e-6, 0.99)
        table.append([t, rl, rv])
    p = ref.make_params(dict(nx=1, ny=1, nz=1, G=-10.0 / 3.0, psi_form="exp", psi0=1.0, rho0=1.0,
                             s_e=1.0, s_nu=1.0, s_q=1.0, s_pi=1.0))
    rl, rv = eos.maxwell(ref.pressure_fn(p), 0.05, 20.0)
    out = {"source": "Maxwell equal-area construction of the oracle's pressure "
                     "p = rho/3 + G psi^2/2 (oracle/eos.py)",
           "carnahan_starling_b4_R1": {"columns": ["T_over_Tc", "rho_L", "rho_V"], "rows": table},
           "exponential_G-10/3": {"rho_L": rl, "rho_V": rv}}
    with open(os.path.join(os.path.dirname(HERE), "lbm_inputs", "coexistence.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
