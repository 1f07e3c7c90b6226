"""Shared helpers of the GPU parity tests: a library context on cuda:0 and
conversion of library tensors into the oracle's block representation."""
import sys

import numpy as np

from oracle import tucker as T


def context():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2306_00632_amd import tk
    tk.lib()  # fails loudly if libtk.so is missing
    return tk.Context(0)


def to_oracle(t) -> T.TuckerSum:
    U, blocks = t.to_host()
    return T.TuckerSum(U, [(c, G, o) for c, G, o in blocks])


def to_oracle_plain(t) -> T.Tucker:
    core, U = t.plain()
    return T.Tucker(core, U)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))
