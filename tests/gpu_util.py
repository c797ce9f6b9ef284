"""Helpers shared by the GPU parity tests (inputs from the seeded generators,
expected values from the oracle; nothing here does field arithmetic)."""
import numpy as np
import torch

from paper_1404_3458_amd import synth


def rand_rows(rows, row_bytes, *key):
    return synth.random_bytes(synth.key(*key), rows * row_bytes).reshape(rows, row_bytes)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def first_diff(a, b):
    d = np.argwhere(a != b)
    return None if len(d) == 0 else (tuple(d[0]), a[tuple(d[0])], b[tuple(d[0])], len(d))
