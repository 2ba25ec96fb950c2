"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np
import torch

from paper_2510_25938_amd import lj

DEV = "cuda"


def announce(msg):
    """Name the case on stdout before a GPU step (flushed)."""
    sys.stdout.write(f"[gpu-case] {msg}\n")
    sys.stdout.flush()


def to_dev(off, xyz):
    batch = lj.ClusterBatch(off, device=DEV)
    return batch, torch.from_numpy(np.ascontiguousarray(xyz)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return None if t is None else t.cpu().numpy()


def host_dict(d):
    torch.cuda.synchronize()
    return {k: (None if v is None else v.cpu().numpy()) for k, v in d.items()}


U32 = 2.0 ** -24
