"""Shared helpers of the GPU parity tests: the HIP library is driven through
the Python binding of the C ABI and compared with the oracle on the same
seeded inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def have_gpu():
    try:
        return torch.cuda.is_available()
    except Exception:
        return False


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()


def rel_err(got, ref):
    ref = np.asarray(ref).reshape(-1)
    got = np.asarray(got).reshape(-1)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def announce(msg):
    print(msg, flush=True)
