"""Error measures and fixtures shared by the GPU parity tests.

Measures (each stated against the FP64 oracle):
  trace     relative error
  lmin      |d lambda| / lambda_max (Weyl-normalised: an eigenvalue moves by at
            most the spectral norm of the perturbation), and the relative error
            where lambda_min > 1e-6 lambda_max
  logdet    absolute error in nats (= relative error of det)
  FIM       e_FIM = |dF|_F / |F|_F (eq:fim_rel_diff)
  blocks    per-voxel |dC|_F / |C|_F over the 10 blocks
"""
from __future__ import annotations

import numpy as np

IU = np.triu_indices(6)
OFF_W = np.where(IU[0] == IU[1], 1.0, 2.0)  # squared-norm weights of the 21 entries


def sym_from21(v):
    v = np.asarray(v)
    F = np.zeros(v.shape[:-1] + (6, 6))
    F[..., IU[0], IU[1]] = v
    F[..., IU[1], IU[0]] = v
    return F


def upper21(F):
    return np.asarray(F)[..., IU[0], IU[1]]


def fro21(v):
    return np.sqrt((np.asarray(v) ** 2 * OFF_W).sum(-1))


def block_rel_err(gpu_blocks, oracle_blocks):
    """gpu_blocks [n,10,21]; oracle_blocks [n,10,6,6] -> per-voxel relative error."""
    ref = upper21(oracle_blocks)
    d = np.sqrt(((gpu_blocks - ref) ** 2 * OFF_W).sum(axis=(-1, -2)))
    n = np.sqrt((ref ** 2 * OFF_W).sum(axis=(-1, -2)))
    return d / np.maximum(n, 1e-300)


def lambda_max(F21):
    return np.linalg.eigvalsh(sym_from21(F21))[..., -1]


def metric_errors(gpu, ref, fim_ref21, cols=("trace", "lmin", "logdet")):
    """Errors per metric column; fim_ref21 [m,21] scales the lmin measure."""
    out = {}
    lmax = np.abs(lambda_max(fim_ref21))
    for c, name in enumerate(cols):
        g, r = gpu[:, c], ref[:, c]
        if name == "trace":
            out["trace_rel"] = np.abs(g - r) / np.abs(r)
        elif name == "lmin":
            out["lmin_weyl"] = np.abs(g - r) / lmax
            well = r > 1e-6 * lmax
            out["lmin_rel"] = np.abs(g[well] - r[well]) / np.abs(r[well])
        elif name == "logdet":
            both_nan = np.isnan(g) & np.isnan(r)
            e = np.abs(g - r)
            e[both_nan] = 0.0
            out["logdet_abs"] = e
    return out


def e_fim(gpu21, ref21):
    return fro21(np.asarray(gpu21) - np.asarray(ref21)) / fro21(ref21)
