"""Torch-facing plan object over the C ABI (device memory and streams only)."""

import torch

from . import _lib

_SHEARLETS = {"meyer": _lib.FFST_SHEARLET_MEYER, "smooth": _lib.FFST_SHEARLET_MEYER_SMOOTH}


class Plan:
    """Spectra and tables for M x N images with J scales on one GPU.

    forward(x):  x (M, N) or (B, M, N) float32 -> (eta, M, N) or (B, eta, M, N)
    adjoint(c):  the reverse shapes; inverse(c) is the same computation.
    With complex_shearlets=True (one-sided spectra) the coefficients are
    complex64 and adjoint(c) returns the real image Re sum_i ... .
    aux picks the auxiliary function v behind the windows: 3 (eq. (v), the
    default), another order k in [1, 10] (C^k) or "inf" (C-infinity).
    Calls are asynchronous on torch's current stream of the plan's device.
    One workspace per batch size is cached on the plan, so calls that may
    run at the same time on different streams need their own `ws`.
    """

    def __init__(self, M, N, J=0, max_scale="max", shearlet="meyer", complex_shearlets=False, aux=3,
                 device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1202_1773_amd needs a ROCm GPU (no CPU path exists)")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._h = None
        with torch.cuda.device(self.device):
            self._h = _lib.ffst_spectra(M, N, J, max_scale, _SHEARLETS[shearlet], complex_shearlets, aux)
        self.M, self.N, self.J, self.eta = _lib.ffst_plan_info(self._h)
        self.max_scale = max_scale
        self.shearlet = shearlet
        self.complex_shearlets = bool(complex_shearlets)
        self.aux = aux
        self.coef_dtype = torch.complex64 if self.complex_shearlets else torch.float32
        self._ws = {}

    # ---------------------------------------------------------------- memory
    def workspace_size(self, batch):
        return _lib.ffst_workspace_size(self._h, batch)

    def workspace(self, batch):
        ws = self._ws.get(batch)
        if ws is None:
            nbytes = max(self.workspace_size(batch), 1)
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self._ws[batch] = ws
        ptr = ws.data_ptr()
        return ptr + (-ptr) % 256

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def _check(self, t, trailing, dtype=torch.float32):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != dtype:
            raise ValueError(f"expected a {dtype} tensor on {self.device}")
        if not t.is_contiguous():
            raise ValueError("expected a contiguous tensor")
        if tuple(t.shape[-len(trailing):]) != trailing:
            raise ValueError(f"expected trailing shape {trailing}, got {tuple(t.shape)}")

    # ------------------------------------------------------------ transforms
    def forward(self, x, out=None, ws=None):
        self._check(x, (self.M, self.N))
        single = x.dim() == 2
        xb = x.reshape(-1, self.M, self.N)
        B = xb.shape[0]
        if out is None:
            out = torch.empty((B, self.eta, self.M, self.N), dtype=self.coef_dtype, device=self.device)
        self._check(out, (self.eta, self.M, self.N), self.coef_dtype)
        if out.numel() != B * self.eta * self.M * self.N:
            raise ValueError("output has the wrong number of elements")
        call = _lib.ffst_forward_complex if self.complex_shearlets else _lib.ffst_forward
        call(self._h, xb.data_ptr(), out.data_ptr(), B, ws if ws is not None else self.workspace(B), self._stream())
        return out.reshape(self.eta, self.M, self.N) if single else out.reshape(B, self.eta, self.M, self.N)

    def adjoint(self, c, out=None, ws=None):
        self._check(c, (self.eta, self.M, self.N), self.coef_dtype)
        single = c.dim() == 3
        cb = c.reshape(-1, self.eta, self.M, self.N)
        B = cb.shape[0]
        if out is None:
            out = torch.empty((B, self.M, self.N), dtype=torch.float32, device=self.device)
        self._check(out, (self.M, self.N))
        if out.numel() != B * self.M * self.N:
            raise ValueError("output has the wrong number of elements")
        call = _lib.ffst_adjoint_complex if self.complex_shearlets else _lib.ffst_adjoint
        call(self._h, cb.data_ptr(), out.data_ptr(), B, ws if ws is not None else self.workspace(B), self._stream())
        return out.reshape(self.M, self.N) if single else out.reshape(B, self.M, self.N)

    def adjoint_sign(self, c, scale, out=None, ws=None):
        """SH*(scale * sign(c)) for a real-shearlet plan; scale is a one-element
        float32 tensor on the plan's device (read by the kernels)."""
        if self.complex_shearlets:
            raise ValueError("adjoint_sign is for real-shearlet plans")
        self._check(c, (self.eta, self.M, self.N))
        if not (isinstance(scale, torch.Tensor) and scale.device == self.device and scale.dtype == torch.float32
                and scale.numel() == 1):
            raise ValueError("scale must be a one-element float32 tensor on the plan's device")
        single = c.dim() == 3
        cb = c.reshape(-1, self.eta, self.M, self.N)
        B = cb.shape[0]
        if out is None:
            out = torch.empty((B, self.M, self.N), dtype=torch.float32, device=self.device)
        self._check(out, (self.M, self.N))
        if out.numel() != B * self.M * self.N:
            raise ValueError("output has the wrong number of elements")
        sc = scale.contiguous()
        _lib.ffst_adjoint_sign(self._h, cb.data_ptr(), out.data_ptr(), B, sc.data_ptr(),
                               ws if ws is not None else self.workspace(B), self._stream())
        return out.reshape(self.M, self.N) if single else out.reshape(B, self.M, self.N)

    def inverse(self, c, out=None, ws=None):
        return self.adjoint(c, out=out, ws=ws)

    # ---------------------------------------------------------------- tuning
    def tuning(self):
        """(nparts, blocks_per_cu) of the plan; 0 means the built-in choice."""
        return _lib.ffst_get_tuning(self._h)

    def set_tuning(self, nparts=0, blocks_per_cu=0, col_values=0, row_block=0, fwd_nparts=0):
        """Launch settings (ffst_tuning in include/ffst.h); 0 keeps a default."""
        _lib.ffst_set_tuning_ex(self._h, nparts, blocks_per_cu, col_values, row_block, fwd_nparts)
        self._ws.clear()

    def tuning_ex(self):
        """All launch settings: dict(nparts, blocks_per_cu, col_values, row_block, fwd_nparts)."""
        return _lib.ffst_get_tuning_ex(self._h)

    def tune(self, x):
        """Autotune the launch settings for forward + adjoint of the images x
        ((M, N) or (B, M, N), float32); returns the best time in ms."""
        self._check(x, (self.M, self.N))
        xb = x.reshape(-1, self.M, self.N)
        B = xb.shape[0]
        saved = self.tuning()
        _lib.ffst_set_tuning(self._h, 8, saved[1])        # largest workspace of any setting
        ws_size = max(self.workspace_size(B), _lib.ffst_workspace_size(self._h, B))
        _lib.ffst_set_tuning(self._h, *saved)
        ws = torch.empty(ws_size + 256, dtype=torch.uint8, device=self.device)
        ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
        c = torch.empty((B, self.eta, self.M, self.N), dtype=self.coef_dtype, device=self.device)
        y = torch.empty_like(xb)
        best = _lib.ffst_tune(self._h, xb.data_ptr(), c.data_ptr(), y.data_ptr(), B, ptr, ws_size, self._stream())
        self._ws.clear()
        return best

    # --------------------------------------------------------------- helpers
    def spectra(self, full_plane=False):
        """The plan's float32 spectra, (eta, M, N/2+1) or (eta, M, N); the
        one-sided spectra of a complex plan exist on the full plane only."""
        cols = self.N if full_plane else self.N // 2 + 1
        dst = torch.empty((self.eta, self.M, cols), dtype=torch.float32, device=self.device)
        torch.cuda.synchronize(self.device)
        _lib.ffst_get_spectra(self._h, dst.data_ptr(), 1 if full_plane else 0)
        return dst

    def scale_shear(self, i):
        """('lowpass' | 'horizontal' | 'vertical' | 'seam', j, k) of plane i;
        its dilation and shear are a = 4^-j and s = k 2^-j (j = -1 for the
        low-pass)."""
        kind, j, k = _lib.ffst_scale_shear(self.J, i)
        return _lib.KIND_NAMES[kind], j, k

    def index(self, kind, j=0, k=0):
        """Plane index of (kind, j, k), kind as returned by scale_shear."""
        code = {v: c for c, v in _lib.KIND_NAMES.items()}[kind]
        return _lib.ffst_shearlet_index(self.J, code, j, k)

    def windows(self):
        """Per spectrum, the first and last column holding a nonzero (half
        plane; for a complex plan a cyclic range of full-plane columns)."""
        return _lib.ffst_plan_windows(self._h, self.eta)

    def close(self):
        if self._h:
            _lib.ffst_destroy(self._h)
            self._h = None
        self._ws.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
