"""Array-namespace shim so the oracle runs unchanged on NumPy or on torch-CPU.

Test infrastructure only. NumPy gives fast float64 runs for the pins, and
the same source in x86 extended precision (np.longdouble arrays, 64-bit
significands) where a comparison needs a reference whose own rounding is far
below FP64's; torch (CPU, float64) gives reverse-mode gradients of the very
same oracle source. Only array plumbing lives here: no arithmetic of the
method.
"""
import numpy as np

try:  # torch is optional for the oracle; only the gradient pins need it
    import torch
except ImportError:  # pragma: no cover
    torch = None


def is_torch(a):
    return torch is not None and isinstance(a, torch.Tensor)


class _NP:
    float64 = np.float64

    @staticmethod
    def sqrt(a):
        return np.sqrt(a)

    @staticmethod
    def stack(xs, axis=0):
        return np.stack(xs, axis=axis)

    @staticmethod
    def take(a, idx, axis):
        return np.take(a, idx, axis=axis)

    @staticmethod
    def moveaxis(a, src, dst):
        return np.moveaxis(a, src, dst)

    @staticmethod
    def inv(a):
        if a.dtype == np.longdouble and np.longdouble != np.float64:
            return _inv_gauss_jordan(a)
        return np.linalg.inv(a)

    @staticmethod
    def matvec(m, v):
        # m: (..., r, c), v: (c, ...) -> (r, ...) with the batch axes trailing
        mv = np.moveaxis(v, 0, -1)[..., None]
        return np.moveaxis((m @ mv)[..., 0], -1, 0)

    @staticmethod
    def amax(a):
        return float(np.max(a))

    @staticmethod
    def zeros_like(a):
        return np.zeros_like(a)

    @staticmethod
    def const(c, like):
        dt = like.dtype if getattr(like, 'dtype', None) == np.longdouble else np.float64
        return np.asarray(c, dtype=dt)


class _TORCH:
    float64 = None if torch is None else torch.float64

    @staticmethod
    def sqrt(a):
        return torch.sqrt(a)

    @staticmethod
    def stack(xs, axis=0):
        return torch.stack(xs, dim=axis)

    @staticmethod
    def take(a, idx, axis):
        return torch.index_select(a, axis, torch.as_tensor(idx, dtype=torch.long))

    @staticmethod
    def moveaxis(a, src, dst):
        return torch.movedim(a, src, dst)

    @staticmethod
    def inv(a):
        return torch.linalg.inv(a)

    @staticmethod
    def matvec(m, v):
        mv = torch.movedim(v, 0, -1).unsqueeze(-1)
        return torch.movedim((m @ mv).squeeze(-1), -1, 0)

    @staticmethod
    def amax(a):
        return float(torch.max(a.detach()))

    @staticmethod
    def zeros_like(a):
        return torch.zeros_like(a)

    @staticmethod
    def const(c, like):
        return torch.as_tensor(c, dtype=like.dtype)


def _inv_gauss_jordan(a):
    """Inverse of every matrix of a stack (..., n, n) by Gauss-Jordan
    elimination with partial pivoting, in the stack's own dtype (NumPy's
    linalg has no extended-precision routines)."""
    n = a.shape[-1]
    aug = np.concatenate([a, np.broadcast_to(np.eye(n, dtype=a.dtype), a.shape)], axis=-1).copy()
    idx = np.indices(a.shape[:-2])
    for k in range(n):
        piv = np.argmax(np.abs(aug[..., k:, k]), axis=-1) + k
        kk = np.full_like(piv, k)
        row_k = aug[(*idx, kk)].copy()
        aug[(*idx, kk)] = aug[(*idx, piv)]
        aug[(*idx, piv)] = row_k
        aug[..., k, :] = aug[..., k, :] / aug[..., k, k:k + 1]
        for i in range(n):
            if i != k:
                aug[..., i, :] = aug[..., i, :] - aug[..., i, k:k + 1] * aug[..., k, :]
    return aug[..., n:]


def ns(a):
    """Namespace for the array type of ``a``."""
    return _TORCH if is_torch(a) else _NP
