"""Shared helpers of the GPU parity tests: device transfer and comparisons."""
import numpy as np
import torch

DEV = "cuda:0"


def dev_bits(words: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(words).view(np.int64)).to(DEV)


def host_bits(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def dev_c128(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.complex128))).to(DEV)


def wrap_phase(d):
    return (d + np.pi) % (2 * np.pi) - np.pi


def assert_logpsi_close(got, ref, rtol=1e-10):
    got, ref = np.asarray(got), np.asarray(ref)
    scale = np.maximum(1.0, np.abs(ref))
    assert np.all(np.abs(got.real - ref.real) <= rtol * scale), np.max(np.abs(got.real - ref.real) / scale)
    assert np.all(np.abs(wrap_phase(got.imag - ref.imag)) <= rtol * scale)


def flush(msg):
    print(msg, flush=True)
