"""Write the lattice pins of the oracle to lattice_pins.json.

Calls only the oracle.  The stored values are regression anchors; the tests
also check each one against a closed form the paper's definitions fix
(partition of unity of the kernel, Eq. kernel; continuum limits of the
pressure and viscosity terms, Alg. 1).

    python tests/golden/make_pins.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402

M = 6            # lattice half-width in sites; support 2h = 4 s fits inside
S = 0.25         # exactly representable spacing, so lattice distances are exact
H = 2 * S


def lattice(m=M, s=S):
    r = np.arange(-m, m + 1, dtype=np.float64) * s
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    centre = int(np.argmin(np.linalg.norm(x, axis=1)))
    return x, centre


def params(nu=0.0, g=(0.0, 0.0, 0.0), m=M, s=S):
    ext = (m + 1) * s
    return {"h": 2 * s, "rho0": 1000.0, "k_pressure": 250.0, "nu": nu, "gravity": g, "dt": 1e-3,
            "domain_lo": (-ext, -ext, -ext), "domain_hi": (ext, ext, ext), "flags": 0}


def lattice_density():
    x, c = lattice()
    n = x.shape[0]
    P = params()
    mass = np.full(n, 1000.0 * S ** 3)
    rho, _ = oracle.density(P, "f64", x, mass, np.zeros(n, np.uint8), np.zeros(n), [c])
    cnt = oracle.neighbors(P, "f64", x, [c])[0][0]
    return rho[0] / 1000.0, int(cnt)


def gradient_factor():
    """Pressure force on the centre of a lattice with p = b x and uniform rho0:
    f = -G V grad p defines G (continuum value 1)."""
    x, c = lattice()
    n = x.shape[0]
    P = params()
    mass = np.full(n, 1000.0 * S ** 3)
    b = 1.0
    p = b * x[:, 0]
    rho = np.full(n, 1000.0)
    f = oracle.forces(P, "f64", x, np.zeros_like(x), mass, np.zeros(n, np.uint8), np.zeros(n),
                      rho, p, None, [c])
    V = S ** 3
    return float(-f[0, 0] / (V * b))


def brookshaw_sum():
    """Viscous force on the centre with v = (x^2, 0, 0), p = 0, rho = rho0,
    nu = 1: f_x = m nu B, continuum B = lap v_x = 2."""
    x, c = lattice()
    n = x.shape[0]
    P = params(nu=1.0)
    mass = np.full(n, 1000.0 * S ** 3)
    v = np.zeros_like(x)
    v[:, 0] = x[:, 0] ** 2
    rho = np.full(n, 1000.0)
    f = oracle.forces(P, "f64", x, v, mass, np.zeros(n, np.uint8), np.zeros(n), rho, np.zeros(n),
                      None, [c])
    return float(f[0, 0] / (mass[0] * 1.0))


def flat_wall_volume():
    """psi_b of the centre particle of a single-layer square wall of spacing s."""
    r = np.arange(-M, M + 1, dtype=np.float64) * S
    X, Y = np.meshgrid(r, r, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1)
    c = int(np.argmin(np.linalg.norm(x, axis=1)))
    n = x.shape[0]
    psi = oracle.boundary_psi(params(), "f64", x, np.full(n, 2, np.uint8), np.zeros(n, np.int32))
    return float(psi[c] / 1000.0 / S ** 3)


def main():
    rho_rel, cnt = lattice_density()
    out = {
        "_source": "written by tests/golden/make_pins.py from the oracle only; h = 2 s, s = 0.25",
        "lattice_density_over_rho0": {"value": rho_rel,
                                      "cite": "Eq. density with m = rho0 s^3; Eq. kernel"},
        "lattice_neighbors_incl_self": {"value": cnt, "cite": "Eq. kernel support 2h, strict r < 2h"},
        "gradient_factor_G": {"value": gradient_factor(),
                              "cite": "Alg. 1 pressure force, symmetric discrete form"},
        "brookshaw_sum_B": {"value": brookshaw_sum(),
                            "cite": "Alg. 1 viscosity force, Brookshaw/Morris form, eps = 0.01 h^2"},
        "flat_wall_Vb_over_s3": {"value": flat_wall_volume(),
                                 "cite": "boundary particle volume, Sec. 3.2 typed particles"},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lattice_pins.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
