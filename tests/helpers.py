"""Shared test plumbing: build the oracle and the HIP context from the same
seeded workload instance, and compare their outputs."""
import copy
import math

import numpy as np
import torch

from oracle.model import Model, Problem
from oracle.stepper import Stepper


def oracle_for(inst, method=None, dt0=None):
    M = Model(Problem(**inst.oracle_kwargs()))
    st = Stepper(M, inst.m0.astype(np.float64), inst.a0, method=method or inst.method, dt0=dt0 or inst.dt0)
    return st


def gpu_for(inst, workspace="torch"):
    from paper_2603_03706_amd import mmcav
    return mmcav.Context.from_instance(inst, workspace=workspace)


def run_oracle(st, T, tol=0.0):
    with torch.no_grad():
        return st.run(T, tol)


def m_err(m_gpu, st):
    return float(np.abs(m_gpu.astype(np.float64) - st.m.numpy()).max())


def rel_a_err(a_gpu, a_ref):
    a_ref = np.asarray(a_ref)
    scale = max(np.abs(a_ref).max(), 1e-300)
    return float(np.abs(np.asarray(a_gpu) - a_ref).max() / scale)


def variant(inst, **kw):
    out = copy.deepcopy(inst)
    for k, v in kw.items():
        setattr(out, k, v)
    return out
