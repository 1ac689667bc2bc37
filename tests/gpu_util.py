"""Helpers for the GPU tests: device selection and oracle-side comparisons."""
import numpy as np
import pytest
import torch


def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to64(t):
    return t.detach().cpu().double().numpy()


def unpack_bits(words, count):
    w = np.asarray(words, dtype=np.uint32)
    bits = np.unpackbits(w.view(np.uint8), bitorder="little")
    return bits[:count]


def say(*a):
    print(*a, flush=True)
