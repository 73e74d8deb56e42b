"""Helpers of the GPU tests: move numpy inputs to the device, print the case."""
import sys

import numpy as np


def dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def announce(*what):
    print("CASE", *what, flush=True)
    sys.stdout.flush()
