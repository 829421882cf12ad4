"""ctypes binding of include/mlp.h: the surrogate network's HIP train/infer
kernels (argument marshalling only; torch supplies device memory and stream)."""
import ctypes

import numpy as np

from . import lb as _lb

NPARAM = 4481
_FP = ctypes.POINTER(ctypes.c_float)
_bound = False


def _bind():
    global _bound
    L = _lb.load_library()
    if _bound:
        return L
    H = ctypes.c_void_p
    sig = {
        "mlp_state_bytes": [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
        "mlp_init": [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(H)],
        "mlp_set_params": [H, _FP],
        "mlp_get_params": [H, _FP],
        "mlp_set_norm": [H, _FP, _FP, ctypes.c_float, ctypes.c_float],
        "mlp_set_data": [H, _FP, _FP, ctypes.c_int32],
        "mlp_loss_grad": [H, _FP, _FP],
        "mlp_train": [H, ctypes.c_int32, ctypes.c_float, _FP],
        "mlp_infer": [H, _FP, ctypes.c_int32, _FP],
        "mlp_destroy": [H],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    _bound = True
    return L


def _f32(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape is not None and a.shape != shape:
        raise ValueError(f"array of shape {a.shape}, expected {shape}")
    return a


def _p(a):
    return a.ctypes.data_as(_FP)


class MLP:
    """3 -> 64 -> 64 -> 1 tanh network on one GPU."""

    def __init__(self, max_rows=4096, device="cuda:0"):
        import torch
        L = _bind()
        self.L = L
        n = ctypes.c_size_t()
        _lb._check(L.mlp_state_bytes(int(max_rows), ctypes.byref(n)))
        self.device = torch.device(device)
        self.state = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self.max_rows = int(max_rows)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            _lb._check(L.mlp_init(ctypes.c_void_p(self.state.data_ptr()), self.state.numel(), self.max_rows,
                                  stream, ctypes.byref(self._h)))

    def set_params(self, theta):
        t = _f32(theta, (NPARAM,))
        _lb._check(self.L.mlp_set_params(self._h, _p(t)))

    def get_params(self):
        t = np.empty(NPARAM, dtype=np.float32)
        _lb._check(self.L.mlp_get_params(self._h, _p(t)))
        return t

    def set_norm(self, in_mean, in_std, out_mean, out_std):
        m = _f32(in_mean, (3,))
        s = _f32(in_std, (3,))
        _lb._check(self.L.mlp_set_norm(self._h, _p(m), _p(s), float(out_mean), float(out_std)))

    def set_data(self, X, y):
        X = _f32(X)
        y = _f32(y)
        if X.ndim != 2 or X.shape[1] != 3 or y.shape != (X.shape[0],):
            raise ValueError("X must be (n, 3) and y (n,)")
        _lb._check(self.L.mlp_set_data(self._h, _p(X), _p(y), X.shape[0]))

    def loss_grad(self):
        loss = ctypes.c_float()
        g = np.empty(NPARAM, dtype=np.float32)
        _lb._check(self.L.mlp_loss_grad(self._h, ctypes.byref(loss), _p(g)))
        return loss.value, g

    def train(self, iters, lr):
        loss = ctypes.c_float()
        _lb._check(self.L.mlp_train(self._h, int(iters), float(lr), ctypes.byref(loss)))
        return loss.value

    def infer(self, X):
        X = _f32(X)
        if X.ndim != 2 or X.shape[1] != 3:
            raise ValueError("X must be (n, 3)")
        y = np.empty(X.shape[0], dtype=np.float32)
        for a in range(0, X.shape[0], self.max_rows):
            b = min(a + self.max_rows, X.shape[0])
            Xc = np.ascontiguousarray(X[a:b])
            yc = np.empty(b - a, dtype=np.float32)
            _lb._check(self.L.mlp_infer(self._h, _p(Xc), b - a, _p(yc)))
            y[a:b] = yc
        return y

    def close(self):
        if self._h:
            self.L.mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
