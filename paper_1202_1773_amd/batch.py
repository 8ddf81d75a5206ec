"""Uneven batches over the C ABI: images of several sizes, one HIP graph
launch per direction (device memory and streams from torch only)."""

import torch

from . import _lib
from .plan import _SHEARLETS


def default_scales(M, N):
    """floor(1/2 log2 max(M, N)) (Sec. 3.1)."""
    return (max(M, N).bit_length() - 1) // 2


class BatchPlan:
    """Plans for a list of image sizes; images of one size share a plan.

    sizes: list of (M, N); J: one int for all, a list (one per image), or
    None for the default of each size. Images and coefficients live in two
    packed float buffers whose layout the library chooses (every size class
    contiguous): pack() / images() / coefficients() move between the packed
    buffers and per-image views. forward / adjoint take and return packed
    buffers; the first call with a given (input, output, workspace) triple
    captures a HIP graph that later calls replay (the library keeps the
    graphs of the eight most recent triples per direction). Pass `out`
    buffers that persist across calls to make every call a replay.
    """

    def __init__(self, sizes, J=None, max_scale="max", shearlet="meyer", complex_shearlets=False, aux=3,
                 device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1202_1773_amd needs a ROCm GPU (no CPU path exists)")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.sizes = [(int(m), int(n)) for m, n in sizes]
        if J is None:
            Js = [0] * len(self.sizes)
        elif isinstance(J, int):
            Js = [J] * len(self.sizes)
        else:
            Js = [int(j) for j in J]
        # resolve the default per image, so equal sizes with an implicit and
        # an explicit default J fall into one class
        self.J = [j if j > 0 else default_scales(m, n) for j, (m, n) in zip(Js, self.sizes)]
        self.etas = [2 ** (j + 2) - 3 for j in self.J]
        self.complex_shearlets = bool(complex_shearlets)
        self.coef_dtype = torch.complex64 if self.complex_shearlets else torch.float32
        self._h = None
        with torch.cuda.device(self.device):
            self._h = _lib.ffst_batch_create([m for m, _ in self.sizes], [n for _, n in self.sizes], self.J,
                                             max_scale, _SHEARLETS[shearlet], complex_shearlets, aux)
        self.count, self.classes = _lib.ffst_batch_info(self._h)
        self.img_off, self.coef_off, self.img_total, self.coef_total = _lib.ffst_batch_layout(self._h, self.count)
        self._ws = None

    # ---------------------------------------------------------------- buffers
    def workspace(self):
        if self._ws is None:
            n = max(_lib.ffst_batch_workspace_size(self._h), 1)
            self._ws = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        ptr = self._ws.data_ptr()
        return ptr + (-ptr) % 256

    def empty_images(self):
        return torch.empty(self.img_total, dtype=torch.float32, device=self.device)

    def empty_coefficients(self):
        n = self.coef_total // 2 if self.complex_shearlets else self.coef_total
        return torch.empty(n, dtype=self.coef_dtype, device=self.device)

    def pack(self, images, out=None):
        """Copy a list of (M_b, N_b) float32 tensors into a packed image buffer."""
        out = self.empty_images() if out is None else out
        for b, img in enumerate(images):
            M, N = self.sizes[b]
            out[self.img_off[b]: self.img_off[b] + M * N].view(M, N).copy_(img)
        return out

    def images(self, packed):
        """Per-image (M_b, N_b) views of a packed image buffer."""
        return [packed[o: o + M * N].view(M, N) for o, (M, N) in zip(self.img_off, self.sizes)]

    def coefficients(self, packed):
        """Per-image (eta_b, M_b, N_b) views of a packed coefficient buffer."""
        div = 2 if self.complex_shearlets else 1
        out = []
        for b, (M, N) in enumerate(self.sizes):
            o = self.coef_off[b] // div
            out.append(packed[o: o + self.etas[b] * M * N].view(self.etas[b], M, N))
        return out

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def _check(self, t, n, dtype):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != dtype:
            raise ValueError(f"expected a {dtype} tensor on {self.device}")
        if not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"expected a contiguous buffer of {n} elements")

    # ------------------------------------------------------------ transforms
    def forward(self, f, out=None):
        self._check(f, self.img_total, torch.float32)
        out = self.empty_coefficients() if out is None else out
        self._check(out, self.coef_total // (2 if self.complex_shearlets else 1), self.coef_dtype)
        _lib.ffst_batch_forward(self._h, f.data_ptr(), out.data_ptr(), self.workspace(), self._stream())
        return out

    def adjoint(self, c, out=None):
        self._check(c, self.coef_total // (2 if self.complex_shearlets else 1), self.coef_dtype)
        out = self.empty_images() if out is None else out
        self._check(out, self.img_total, torch.float32)
        _lib.ffst_batch_adjoint(self._h, c.data_ptr(), out.data_ptr(), self.workspace(), self._stream())
        return out

    def inverse(self, c, out=None):
        return self.adjoint(c, out=out)

    def tune(self, f):
        """Autotune every size class on the packed images f (drops the graphs)."""
        self._check(f, self.img_total, torch.float32)
        c = self.empty_coefficients()
        y = self.empty_images()
        _lib.ffst_batch_tune(self._h, f.data_ptr(), c.data_ptr(), y.data_ptr(), self.workspace(), self._stream())

    def class_tuning(self):
        """Per size class: dict(M, N, J, nparts, blocks_per_cu, col_values, row_block, fwd_nparts)."""
        out = []
        for c in range(self.classes):
            h = _lib.ffst_batch_class(self._h, c)[0]
            M, N, J, _ = _lib.ffst_plan_info(h)
            out.append(dict(M=M, N=N, J=J, **_lib.ffst_get_tuning_ex(h)))
        return out

    def close(self):
        if self._h:
            _lib.ffst_batch_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
