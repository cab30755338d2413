"""Argument checks of the Python binding that need no GPU: host outputs must
be writable contiguous float64 arrays of the right size (the library writes
into their memory), and host inputs of the wrong size are refused before any
library call."""
import numpy as np
import pytest
import torch

import paper_2410_03148_amd as P


def test_host_output_checks():
    n = 27
    good = np.zeros(n)
    p, dev, keep = P._arg(good, n, out=True)
    assert dev == 0 and keep is good
    for bad in (np.zeros(n, dtype=np.float32), np.zeros(n + 1), np.zeros((n, 2))[:, 0], [0.0] * n):
        with pytest.raises(ValueError):
            P._arg(bad, n, out=True)
    ro = np.zeros(n)
    ro.flags.writeable = False
    with pytest.raises(ValueError):
        P._arg(ro, n, out=True)
    # CPU tensors: float64 contiguous outputs are written in place, others refused
    t = torch.zeros(n, dtype=torch.float64)
    p, dev, keep = P._arg(t, n, out=True)
    assert dev == 0 and keep.ctypes.data == t.data_ptr()
    for bad in (torch.zeros(n, dtype=torch.float32), torch.zeros(2 * n, dtype=torch.float64)[::2],
                torch.zeros(n - 1, dtype=torch.float64)):
        with pytest.raises(ValueError):
            P._arg(bad, n, out=True)


def test_host_input_checks():
    n = 8
    p, dev, keep = P._arg(np.arange(n, dtype=np.float32), n)
    assert dev == 0 and keep.dtype == np.float64 and np.array_equal(keep, np.arange(n))
    p, dev, keep = P._arg(torch.arange(n, dtype=torch.float32), n)
    assert keep.dtype == np.float64
    with pytest.raises(ValueError):
        P._arg(np.zeros(n + 1), n)


def test_autograd_class_is_cached():
    assert P.Homogenise is P.Homogenise
