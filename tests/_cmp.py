"""Comparison helpers shared by the parity tests.

Error norms (the tolerances are the ones the hot path is held to):
  density   max_i |rho - rho_ref| / rho_ref
  force     max_i |f - f_ref| / max(|f_ref_i|, m g)     (m g floor: a resting
            particle's net SPH force is ~ its weight, so plain relative error
            is unbounded where forces cancel)
  wrench    |dF| / max(|F_ref|, rho0 g V),  |dT| / max(|T_ref|, rho0 g V L)
"""
import numpy as np

G = 9.81


def rel_density(rho, ref):
    return float(np.max(np.abs(rho - ref) / np.abs(ref))) if ref.size else 0.0


def rel_force(f, ref, floor):
    if ref.size == 0:
        return 0.0
    den = np.maximum(np.linalg.norm(ref, axis=1), floor)
    return float(np.max(np.linalg.norm(f - ref, axis=1) / den))


def rel_vec(a, ref, floor):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(ref)) / max(np.linalg.norm(ref), floor))


def ulp32(x):
    x = np.abs(np.asarray(x, np.float64)).astype(np.float32)
    return (np.nextafter(x, np.float32(np.inf)) - x).astype(np.float64)


def csr_lists(counts, offs, ids, targets):
    return {int(t): ids[offs[t]:offs[t] + counts[t]].tolist() for t in targets}
