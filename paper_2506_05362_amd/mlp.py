"""Python binding of the surrogate-network C ABI in include/pd_mlp.h.

Marshalling only: forward, backward and Adam run in libpd_mlp.so (BF16 matrix
cores, FP32 accumulation).  Inputs and outputs are PyTorch device tensors; the
network runs on its own PyTorch stream.  There is no fallback when the library
is missing.
"""
from __future__ import annotations

import atexit
import sys
import ctypes as C
import weakref
import os
from typing import Optional, Sequence

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpd_mlp.so")
P = C.c_void_p


def load_library(path: str = _LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build()")
    import torch  # noqa: F401  (bind to PyTorch's HIP runtime, see pd.py)
    L = C.CDLL(path)
    from .pd import ALLOC_FN, FREE_FN
    L.pdm_create.argtypes = [C.POINTER(P), P, C.c_int32, C.c_int64, ALLOC_FN, FREE_FN, P, P]
    L.pdm_param_count.argtypes = [P]
    L.pdm_param_count.restype = C.c_int64
    L.pdm_set_params.argtypes = [P, P, C.c_int64]
    L.pdm_get_params.argtypes = [P, P, C.c_int64]
    L.pdm_set_adam.argtypes = [P, C.c_float, C.c_float, C.c_float, C.c_float]
    L.pdm_forward.argtypes = [P, P, C.c_int64, P]
    L.pdm_set_inference.argtypes = [P, C.c_int32]
    L.pdm_gradients.argtypes = [P, P, P, C.c_int64, C.POINTER(C.c_float), P]
    L.pdm_train_step.argtypes = [P, P, P, C.c_int64, C.c_float, C.POINTER(C.c_float)]
    L.pdm_destroy.argtypes = [P]
    L.pdm_last_error.argtypes = [P]
    L.pdm_last_error.restype = C.c_char_p
    for name in ["pdm_create", "pdm_set_params", "pdm_get_params", "pdm_set_adam", "pdm_forward",
                 "pdm_gradients", "pdm_train_step", "pdm_set_inference"]:
        getattr(L, name).restype = C.c_int32
    return L


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


class MLPError(RuntimeError):
    pass


# networks still open at interpreter exit are destroyed by an exit hook, while
# the HIP runtime is still up
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_nets():
    for net in list(_LIVE):
        try:
            net.close()
        except Exception:
            pass


class Net:
    def __init__(self, dims: Sequence[int], max_batch: int = 4096, stream=None):
        import torch
        self.torch = torch
        self.dims = [int(d) for d in dims]
        self.stream = stream if stream is not None else torch.cuda.Stream()
        d = np.array(self.dims, dtype=np.int32)
        h = P()
        # device buffers come from PyTorch's caching allocator, on this network's stream
        from .pd import ALLOC_FN, FREE_FN
        dev = torch.cuda.current_device()

        def _alloc(nbytes, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, self.stream)
            except Exception:  # out of memory -> NULL -> PD_ERR_OOM
                return None

        def _free(ptr, user):
            cuda = getattr(torch, "cuda", None)
            if cuda is not None:
                cuda.caching_allocator_delete(int(ptr))

        self._alloc, self._free = ALLOC_FN(_alloc), FREE_FN(_free)
        st = lib().pdm_create(C.byref(h), d.ctypes.data_as(P), len(self.dims), int(max_batch),
                              self._alloc, self._free, None, P(self.stream.cuda_stream))
        self.h = h
        _LIVE.add(self)
        self.max_batch = int(max_batch)
        self._check(st)
        self.n_params = int(lib().pdm_param_count(self.h))

    def _check(self, st):
        if st != 0:
            raise MLPError(f"{lib().pdm_last_error(self.h).decode()} (status {st})")

    def _dev(self, t, cols):
        t = t.to(device="cuda", dtype=self.torch.float32).contiguous()
        assert t.dim() == 2 and t.shape[1] == cols
        return t

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._check(lib().pdm_set_params(self.h, p.ctypes.data_as(P), p.size))

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.n_params, dtype=np.float32)
        self._check(lib().pdm_get_params(self.h, p.ctypes.data_as(P), p.size))
        return p

    def set_adam(self, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        self._check(lib().pdm_set_adam(self.h, beta1, beta2, eps, weight_decay))

    def set_inference(self, fused: bool):
        self._check(lib().pdm_set_inference(self.h, 1 if fused else 0))

    def forward(self, x):
        x = self._dev(x, self.dims[0])
        y = self.torch.empty((x.shape[0], self.dims[-1]), device="cuda", dtype=self.torch.float32)
        self.torch.cuda.current_stream().synchronize()
        self._check(lib().pdm_forward(self.h, P(x.data_ptr()), x.shape[0], P(y.data_ptr())))
        return y

    def gradients(self, x, y):
        x, y = self._dev(x, self.dims[0]), self._dev(y, self.dims[-1])
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_float()
        self.torch.cuda.current_stream().synchronize()
        self._check(lib().pdm_gradients(self.h, P(x.data_ptr()), P(y.data_ptr()), x.shape[0],
                                        C.byref(loss), g.ctypes.data_as(P)))
        return float(loss.value), g

    def train_step(self, x, y, lr: float, want_loss: bool = True) -> Optional[float]:
        loss = C.c_float()
        self._check(lib().pdm_train_step(self.h, P(x.data_ptr()), P(y.data_ptr()), x.shape[0], lr,
                                         C.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None

    def close(self):
        if getattr(self, "h", None):
            lib().pdm_destroy(self.h)
            self.h = None
        _LIVE.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # during interpreter teardown the HIP runtime may already be gone: the
        # exit hook closed every context that was still open before that (the
        # check is bound at definition, since module globals may be cleared by then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
