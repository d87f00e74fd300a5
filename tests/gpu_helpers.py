"""Shared helpers of the GPU parity tests (host-side marshalling only)."""
import numpy as np
import torch

from paper_1806_00082_amd import inputs

HB = inputs.HBAR_EVFS


def dev():
    return torch.device("cuda:0")


def normwise(got, ref):
    """max |got - ref| / max |ref| per potential (first axis), then the max over the batch."""
    got = np.asarray(got, dtype=np.float64).reshape(got.shape[0], -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], -1)
    err = np.abs(got - ref).max(axis=1)
    scale = np.abs(ref).max(axis=1)
    scale[scale == 0] = 1.0
    return float((err / scale).max())


def to_np(t):
    return t.detach().cpu().numpy()


def as_u32(t):
    return to_np(t).view(np.uint32)


def as_u64(t):
    return to_np(t).view(np.uint64)


def host_tables_to_device(tables):
    g, n0, thr, cdf = tables
    d = dev()
    return (torch.from_numpy(np.ascontiguousarray(n0).view(np.int32)).to(d),
            torch.from_numpy(np.ascontiguousarray(thr).view(np.int32)).to(d),
            torch.from_numpy(np.ascontiguousarray(cdf).view(np.int64)).to(d))


def assert_particles_equal(gpu_view, host_view, what=""):
    assert set(gpu_view) == set(host_view)
    for k in host_view:
        a, b = gpu_view[k], host_view[k]
        assert a.shape == b.shape, (what, k, a.shape, b.shape)
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{what}: field {k} differs at {len(bad)} slots, first {bad[:5]}: "
                                 f"gpu {a[bad[:5]]} oracle {b[bad[:5]]}")
