"""Helpers shared by the GPU parity tests: build the GPU hierarchy and the oracle
hierarchy of the same seeded domain with the same parameters."""
import numpy as np
import torch

import lsmg_inputs as I
import oracle
from paper_1902_07029_amd import lsmg

LEVELSETS = {"disk": I.disk, "star": I.star, "torus": I.torus, "paper3": I.paper_circle, "paper4": I.paper_square}
DIM = {"disk": 2, "star": 2, "torus": 3, "paper3": 2, "paper4": 2}
# the paper's Tests 3 and 4 live on their own box
BOX = {"paper3": I.PAPER_BOX, "paper4": I.PAPER_BOX}


def oracle_params(p):
    return dict(a=p.a, d=p.d, m_s=p.m_s, m_c=p.m_c, alpha=p.alpha, beta=p.beta, tau_s=p.tau_s, nu1=p.nu1,
                nu2=p.nu2, ghost_c_new=p.ghost_c_new, band_steps=p.band_steps, ghost_sweeps=p.ghost_sweeps,
                ghost_sweeps_coarse=p.ghost_sweeps_coarse, sweeps_lambda=p.sweeps_lambda, gamma=p.cycle_gamma,
                fmg=p.fmg, krylov_m=p.krylov_m)


def pair(kind, n, coarsest, phi=None, **params):
    dim = DIM[kind]
    if phi is None:
        phi = LEVELSETS[kind](n)
    lo, hi = BOX.get(kind, (-1.0, 1.0))
    p = lsmg.default_params(coarsest_n=coarsest, **params)
    H = lsmg.Hierarchy(torch.from_numpy(phi), dim, n, lo, hi, params=p)
    O = oracle.Hierarchy(phi, dim, n, lo, hi, coarsest_n=coarsest, params=oracle_params(H.params), bc=H.params.bc)
    return H, O


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    scale = np.max(np.abs(b)) if b.size else 0.0
    if scale == 0.0:
        return float(np.max(np.abs(a))) if a.size else 0.0
    return float(np.max(np.abs(a - b)) / scale)


def random_state(O, l, rng):
    na = O.level_info(l)["na"]
    return np.concatenate([rng.uniform(0.0, 1.0, na), rng.uniform(0.5, 1.5, na)])


def say(msg):
    print(msg, flush=True)
