"""Thin ctypes binding of the warm-start surrogate in ``libpic.so``
(include/surrogate.h).  Argument marshalling only: features, convolutions,
loss, gradients and Adam run in the library's HIP kernels; PyTorch provides
the device workspace, the stream and the caller's tensors."""
import ctypes as C

import numpy as np

from . import pic

LAYERS = [(16, 64), (64, 64), (64, 64), (64, 64), (64, 64), (64, 39)]
KS = 5
N_WEIGHTS = sum(ci * co * KS for ci, co in LAYERS)
N_BIASES = sum(co for _, co in LAYERS)
N_OUT = LAYERS[-1][1]

SYMBOLS = ["sur_workspace_size", "sur_create", "sur_set_weights", "sur_get_weights", "sur_get_grads",
           "sur_forward", "sur_forward_noalloc", "sur_train_step", "sur_densities", "sur_state", "sur_last_error",
           "sur_destroy"]

_bound = False


def lib():
    global _bound
    L = pic.lib()
    if not _bound:
        P, i, d, f = C.c_void_p, C.c_int, C.c_double, C.c_float
        sig = {
            "sur_workspace_size": ([i, i, C.POINTER(C.c_size_t)], i),
            "sur_create": ([i, i, P, C.c_size_t, P, C.c_uint32, C.POINTER(P)], i),
            "sur_set_weights": ([P, P, P], i),
            "sur_get_weights": ([P, P, P], i),
            "sur_get_grads": ([P, P, P], i),
            "sur_forward": ([P, P, i, P], i),
            "sur_forward_noalloc": ([P, P, i, P], i),
            "sur_train_step": ([P, P, P, i, f, C.POINTER(d)], i),
            "sur_densities": ([P, P, P, i, P], i),
            "sur_state": ([P, P, P, i, P], i),
            "sur_last_error": ([], C.c_char_p),
            "sur_destroy": ([P], None),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _bound = True
    return L


def _check(rc):
    if rc != pic.PIC_OK:
        raise pic.PicError(rc, lib().sur_last_error().decode(errors="replace"))


def workspace_size(max_batch, cells):
    n = C.c_size_t()
    _check(lib().sur_workspace_size(max_batch, cells, C.byref(n)))
    return n.value


def pack(W, b):
    """Lists of per-layer W [Cout][Cin][5] and b [Cout] -> packed FP32 arrays."""
    w = np.concatenate([np.asarray(x, np.float32).reshape(-1) for x in W])
    bb = np.concatenate([np.asarray(x, np.float32).reshape(-1) for x in b])
    assert w.size == N_WEIGHTS and bb.size == N_BIASES
    return np.ascontiguousarray(w), np.ascontiguousarray(bb)


def unpack(w, b):
    W, B, o, ob = [], [], 0, 0
    for ci, co in LAYERS:
        W.append(w[o:o + ci * co * KS].reshape(co, ci, KS))
        B.append(b[ob:ob + co])
        o += ci * co * KS
        ob += co
    return W, B


class Surrogate:
    """The surrogate network on one GPU (batches of up to max_batch samples of
    `cells` positions)."""

    def __init__(self, max_batch, cells=2048, seed=0, device="cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm GPU visible: the surrogate runs only on the GPU")
        self.device = torch.device(device)
        self.max_batch, self.cells = max_batch, cells
        nbytes = workspace_size(max_batch, cells)
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().sur_create(max_batch, cells, C.c_void_p(self.ws.data_ptr()), nbytes,
                                C.c_void_p(self.stream.cuda_stream), seed, C.byref(h)))
        self.h = h
        self._lib = lib()      # kept for close() at interpreter exit, when module globals may be gone

    def close(self):
        """Release the handle (the workspace tensor is released with the object)."""
        if getattr(self, "h", None) is not None and self.h.value:
            self.stream.synchronize()
            self._lib.sur_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _params(self, params):
        import torch
        p = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
        if p.dim() != 2 or p.shape[1] != 4 or not 1 <= p.shape[0] <= self.max_batch:
            raise ValueError("params must be [B, 4] with 1 <= B <= %d" % self.max_batch)
        return p

    def set_weights(self, W, b):
        w, bb = pack(W, b)
        _check(lib().sur_set_weights(self.h, w.ctypes.data_as(C.c_void_p), bb.ctypes.data_as(C.c_void_p)))

    def weights(self):
        w = np.empty(N_WEIGHTS, np.float32)
        b = np.empty(N_BIASES, np.float32)
        _check(lib().sur_get_weights(self.h, w.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p)))
        return unpack(w, b)

    def grads(self):
        w = np.empty(N_WEIGHTS, np.float32)
        b = np.empty(N_BIASES, np.float32)
        _check(lib().sur_get_grads(self.h, w.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p)))
        return unpack(w, b)

    def forward(self, params, out=None):
        """params [B, 4] (Gamma, T_c K, V, n_g) -> [B, N_OUT, cells] float32 on the GPU."""
        import torch
        p = self._params(params)
        if out is None:
            out = torch.empty((p.shape[0], N_OUT, self.cells), dtype=torch.float32, device=self.device)
        _check(lib().sur_forward(self.h, C.c_void_p(p.data_ptr()), p.shape[0], C.c_void_p(out.data_ptr())))
        return out

    def train_step(self, params, target, lr, want_loss=True):
        import torch
        p = self._params(params)
        t = torch.as_tensor(target, dtype=torch.float32).to(self.device).contiguous()
        if tuple(t.shape) != (p.shape[0], N_OUT, self.cells):
            raise ValueError("target must be [B, %d, cells]" % N_OUT)
        loss = C.c_double()
        _check(lib().sur_train_step(self.h, C.c_void_p(p.data_ptr()), C.c_void_p(t.data_ptr()), p.shape[0],
                                    float(lr), C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def densities(self, params, n0):
        """Warm-start densities [B, 2, cells] float64 (n_e, n_i in m^-3)."""
        import torch
        p = self._params(params)
        n0 = torch.as_tensor(n0, dtype=torch.float64).to(self.device).reshape(-1).contiguous()
        if n0.shape[0] != p.shape[0]:
            raise ValueError("one n0 per sample")
        out = torch.empty((p.shape[0], 2, self.cells), dtype=torch.float64, device=self.device)
        _check(lib().sur_densities(self.h, C.c_void_p(p.data_ptr()), C.c_void_p(n0.data_ptr()), p.shape[0],
                                   C.c_void_p(out.data_ptr())))
        return out

    def state(self, params, n0):
        """Warm-start state [B, 39, cells] float64 for pic_init_from_state
        (densities, potential, velocity quantiles in m/s)."""
        import torch
        p = self._params(params)
        n0 = torch.as_tensor(n0, dtype=torch.float64).to(self.device).reshape(-1).contiguous()
        if n0.shape[0] != p.shape[0]:
            raise ValueError("one n0 per sample")
        out = torch.empty((p.shape[0], N_OUT, self.cells), dtype=torch.float64, device=self.device)
        _check(lib().sur_state(self.h, C.c_void_p(p.data_ptr()), C.c_void_p(n0.data_ptr()), p.shape[0],
                               C.c_void_p(out.data_ptr())))
        return out
