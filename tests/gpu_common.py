"""Shared helpers for the GPU tests (seeded systems, device handles)."""
import functools
import sys

import numpy as np
import pytest

import sci_inputs as si

H_TOL = 1e-12   # Ha, per matrix element
E_TOL = 1e-10   # Ha, energy
G_TOL = 1e-10   # per gradient component


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_2604_15768_amd as sci  # fails loudly when the library is not built
    return sci


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def system(name):
    return si.make_system(si.WORKLOADS[name])


@functools.lru_cache(maxsize=None)
def ham(name):
    sci = require_gpu()
    s = system(name)
    return sci.Ham(s.n_orb, s.n_alpha, s.n_beta, s.h1, s.eri)


def pick_sources(n, k, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    picks = set([0, n - 1])
    picks.update(rng.choice(n, size=min(n, k) - 2, replace=False).tolist())
    return np.array(sorted(picks), dtype=np.int64)
