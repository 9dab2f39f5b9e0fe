"""Helpers for the GPU parity tests: device buffers and oracle-side reshaping."""
import sys

import numpy as np


def say(*a):
    """Name the case before each GPU step (flushed, so a fault log shows it)."""
    print(*a, flush=True)
    sys.stdout.flush()


def upload(x, dev, stride=None):
    """x [beam, t, chan] uint8 -> device [beam, t, stride] (padding bytes 0x5A)."""
    import torch
    nb, nt, nc = x.shape
    stride = stride or (nc + 15) // 16 * 16
    buf = torch.full((nb, nt, stride), 0x5A, dtype=torch.uint8, device=dev)
    buf[:, :, :nc] = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    return buf


def sums_buffers(nbeam, nsub, nchan, dev):
    import torch
    ncell = nsub * nchan
    npair = nbeam * (nbeam + 1) // 2
    sx = torch.full((nbeam, ncell), -7, dtype=torch.int32, device=dev)
    sxy = torch.full((npair, ncell), -7, dtype=torch.int32, device=dev)
    cnt = torch.full((max(nsub, 1),), -7, dtype=torch.int32, device=dev)
    return sx, sxy, cnt


def packed_oracle_sums(S, S2):
    """Oracle S [k, j, b], S2 [k, j, a, b] -> SoA (sum_x [b][cell], sum_xy [pair][cell])
    with pair(a, b) in row-major upper-triangle order."""
    nsub, nchan, nb = S.shape
    ncell = nsub * nchan
    iu = np.triu_indices(nb)
    sx = S.reshape(ncell, nb).T
    sxy = S2.reshape(ncell, nb, nb)[:, iu[0], iu[1]].T
    return sx, sxy


def eig_buffers(nbeam, ncell, dev, with_vectors=True):
    import torch
    stat = torch.full((ncell,), -1.0, dtype=torch.float64, device=dev)
    status = torch.full((ncell,), 0xEE, dtype=torch.uint8, device=dev)
    ev = torch.full((nbeam, ncell), -9.0, dtype=torch.float32, device=dev) if with_vectors else None
    v1 = torch.full((nbeam, ncell), -9.0, dtype=torch.float32, device=dev) if with_vectors else None
    return stat, status, ev, v1
