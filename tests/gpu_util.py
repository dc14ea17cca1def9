"""Shared helpers of the GPU tests: seeded inputs, both sides built from them."""
import numpy as np

import oracle
from paper_2202_07388_amd import qdw
from paper_2202_07388_amd import synthetic as syn


def make_pair(dims, m0, csw, eps=0.3, seed=7388, bc=-1, eps_u1=0.1):
    su3, th = syn.gauge_field(dims, eps, eps_u1, seed)
    gop = qdw.Op(dims, su3, th, m0, csw, bc)
    oop = oracle.Operator(dims, su3, th, m0, csw, bc)
    return gop, oop, su3, th


def rel(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxrel(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.abs(a - b).max() / np.abs(b).max())
