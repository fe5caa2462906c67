"""Python face of libspfel: argument marshalling only.

Each function checks dtypes/devices/contiguity, passes raw device pointers
and the current HIP stream to the C ABI of the same name, and returns the
output tensors.  Every step of slicing, matching and merging runs in the
library's kernels; PyTorch only owns the memory and the stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import check

REAL, COMPLEX = 0, 1
F32, BF16 = 0, 1
MATCH_FP32, MATCH_BF16_RESCORE8 = 0, 1
MERGE_ACCUMULATE, MERGE_DEFER = 1, 2
PHASE_ER, PHASE_HIO = 0, 1


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _p(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _need(t: torch.Tensor, name: str, dtype, device=None, shape=None) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Plan:
    """Slicing/merging plan for an N^3 model (N odd) on one GPU."""

    def __init__(self, n_model: int, kernel_width: int = 6, upsampfac: float = 2.0,
                 beta_over_w: float = 2.30, domain: int = REAL, device=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.n_model = n_model
        self.domain = domain
        self.kernel_width = kernel_width
        h = ctypes.c_void_p()
        check(_lib.lib().spfel_plan_create(ctypes.byref(h), n_model, kernel_width, upsampfac,
                                           beta_over_w, domain, dev.index))
        self._h = h

    @property
    def handle(self):
        return self._h

    @property
    def cdtype(self):
        return torch.complex64 if self.domain == COMPLEX else torch.float32

    def info(self):
        nf = ctypes.c_int()
        nb = ctypes.c_size_t()
        check(_lib.lib().spfel_plan_info(self._h, ctypes.byref(nf), ctypes.byref(nb)))
        return nf.value, nb.value

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value is not None:
            check(_lib.lib().spfel_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_detector(self, det_q: torch.Tensor) -> None:
        """Register the detector template (P, 3); later ``slice`` and
        ``merge_adjoint`` calls without ``det_q`` use its tiled kernels."""
        _need(det_q, "det_q", torch.float32, self.device)
        if det_q.dim() != 2 or det_q.shape[1] != 3:
            raise ValueError("det_q must be (P, 3)")
        check(_lib.lib().spfel_set_detector(self._h, _p(det_q), det_q.shape[0],
                                            _stream(self.device)))
        self.n_det_points = det_q.shape[0]

    def _detector(self, det_q):
        if det_q is None:
            P = getattr(self, "n_det_points", 0)
            if P == 0:
                raise ValueError("no det_q given and no detector registered")
            return None, P
        _need(det_q, "det_q", torch.float32, self.device)
        if det_q.dim() != 2 or det_q.shape[1] != 3:
            raise ValueError("det_q must be (P, 3)")
        return det_q, det_q.shape[0]

    def set_model(self, model: torch.Tensor) -> None:
        N = self.n_model
        _need(model, "model", self.cdtype, self.device, (N, N, N))
        check(_lib.lib().spfel_set_model(self._h, _p(model), _stream(self.device)))

    def slice(self, quats: torch.Tensor, det_q: Optional[torch.Tensor] = None,
              norms: bool = False):
        """Model images at orientations ``quats`` (M,4) and detector points
        ``det_q`` (P,3) (None: the registered detector).  Returns (slices,
        squared norms or None)."""
        _need(quats, "quats", torch.float32, self.device)
        if quats.dim() != 2 or quats.shape[1] != 4:
            raise ValueError("quats must be (M, 4)")
        det_q, P = self._detector(det_q)
        M = quats.shape[0]
        s = torch.empty((M, P), dtype=self.cdtype, device=self.device)
        sn = torch.empty((M,), dtype=torch.float32, device=self.device) if norms else None
        check(_lib.lib().spfel_slice(self._h, _p(quats), M, _p(det_q), P, _p(s), _p(sn),
                                     _stream(self.device)))
        return s, sn

    def merge_adjoint(self, quats: torch.Tensor, det_q: Optional[torch.Tensor],
                      values: torch.Tensor, weights: Optional[torch.Tensor] = None,
                      out: Optional[torch.Tensor] = None, flags: int = 0) -> Optional[torch.Tensor]:
        """Type-1 adjoint of the values (n_img, P) at the images' points,
        onto N^3 modes (det_q None: the registered detector).  With
        MERGE_DEFER only spreads (returns None)."""
        _need(quats, "quats", torch.float32, self.device)
        det_q, P = self._detector(det_q)
        n_img = quats.shape[0]
        _need(values, "values", self.cdtype, self.device, (n_img, P))
        if weights is not None:
            _need(weights, "weights", torch.float32, self.device, (n_img, P))
        N = self.n_model
        if out is None and not (flags & MERGE_DEFER):
            out = torch.empty((N, N, N), dtype=self.cdtype, device=self.device)
        elif out is not None:
            _need(out, "out", self.cdtype, self.device, (N, N, N))
        check(_lib.lib().spfel_merge_adjoint(self._h, _p(quats), n_img, _p(det_q), P, _p(values),
                                             _p(weights), _p(out), flags, _stream(self.device)))
        return out

    def orient(self, quats: torch.Tensor, images, best_idx: torch.Tensor,
               best_dist: torch.Tensor, mode: int = MATCH_FP32, chunk: int = 2048,
               det_q: Optional[torch.Tensor] = None, overlap: bool = True,
               flags: Optional[torch.Tensor] = None) -> tuple:
        """Slice ``quats`` in chunks and match the images against each chunk
        (the slicing of one chunk may overlap the matching of the previous on
        a second stream); folds into (best_idx, best_dist) in place.
        ``images``: ``ImagesF32`` (FP32 mode) or ``ImagesBF16`` (BF16 mode)."""
        if self.domain != REAL:
            raise ValueError("orient needs a REAL plan")
        _need(quats, "quats", torch.float32, self.device)
        det_q, P = self._detector(det_q)
        if mode == MATCH_FP32:
            if not isinstance(images, ImagesF32):
                raise TypeError("FP32 mode takes ImagesF32")
            ops_img, n2, f32, err, centre = images.x, images.norm2, None, None, None
        else:
            if not isinstance(images, ImagesBF16):
                raise TypeError("BF16 mode takes ImagesBF16")
            ops_img, n2, f32, err, centre = images.b16, images.norm2, images.x, images.err, images.centre
        n_img = ops_img.shape[0]
        if ops_img.shape[1] != P:
            raise ValueError("images and detector disagree on P")
        _need(best_idx, "best_idx", torch.int32, self.device, (n_img,))
        _need(best_dist, "best_dist", torch.float32, self.device, (n_img,))
        if flags is not None:
            _need(flags, "flags", torch.int32, self.device, (n_img,))
        M = quats.shape[0]
        c = max(1, min(chunk, M))
        need = int(_lib.lib().spfel_orient_workspace_bytes(c, n_img, P, mode))
        main = torch.cuda.current_stream(self.device)
        aux = main
        if overlap:
            if getattr(self, "_aux", None) is None:
                self._aux = torch.cuda.Stream(device=self.device)
            aux = self._aux
        ws = getattr(self, "_orient_ws", None)
        if ws is None or ws.numel() < need:
            if ws is not None:
                ws.record_stream(aux)
            ws = torch.empty((need,), dtype=torch.uint8, device=self.device)
            self._orient_ws = ws
        ws.record_stream(aux)
        check(_lib.lib().spfel_orient(self._h, _p(quats), M, _p(det_q), P, _p(images.g),
                                      _p(ops_img), _p(n2),
                                      _p(f32), _p(err), _p(centre), n_img, mode, c,
                                      _p(best_idx), _p(best_dist), _p(flags), _p(ws), ws.numel(),
                                      main.cuda_stream, aux.cuda_stream))
        return best_idx, best_dist

    def weighted_residual(self, slices: torch.Tensor, images: torch.Tensor,
                          weights: Optional[torch.Tensor] = None, scale: float = 1.0,
                          residual: bool = True, loss: Optional[torch.Tensor] = None,
                          scale_dev: Optional[torch.Tensor] = None):
        """residual = scale * scale_dev * w (s - d) (or None) and
        loss += sum w |s - d|^2 (a float64 device scalar, created if not
        given).  ``scale_dev``: optional float32 device scalar."""
        _need(slices, "slices", self.cdtype, self.device)
        _need(images, "images", self.cdtype, self.device, tuple(slices.shape))
        if weights is not None:
            _need(weights, "weights", torch.float32, self.device, tuple(slices.shape))
        if scale_dev is not None:
            _need(scale_dev, "scale_dev", torch.float32, self.device)
            if scale_dev.numel() != 1:
                raise ValueError("scale_dev must hold one value")
        if loss is None:
            loss = torch.zeros((), dtype=torch.float64, device=self.device)
        else:
            _need(loss, "loss", torch.float64, self.device)
        r = torch.empty_like(slices) if residual else None
        check(_lib.lib().spfel_weighted_residual(self._h, _p(slices), _p(images), _p(weights),
                                                 slices.numel(), float(scale), _p(scale_dev),
                                                 _p(r), _p(loss), _stream(self.device)))
        return r, loss


def row_norm2(x: torch.Tensor) -> torch.Tensor:
    """Squared norms of the rows of a (rows, cols) float32/bfloat16 matrix."""
    if x.dtype not in (torch.float32, torch.bfloat16):
        raise TypeError("row_norm2 takes float32 or bfloat16")
    _need(x, "x", x.dtype)
    if x.dim() != 2:
        raise ValueError("row_norm2 takes a matrix")
    out = torch.empty((x.shape[0],), dtype=torch.float32, device=x.device)
    check(_lib.lib().spfel_row_norm2(_p(x), BF16 if x.dtype == torch.bfloat16 else F32,
                                     x.shape[0], x.shape[1], _p(out), _stream(x.device)))
    return out


def column_mean(x: torch.Tensor, round_to_integer: bool = True) -> torch.Tensor:
    """Per-column mean of a (rows, cols) float32 matrix (rounded to integers
    by default): the centre of the BF16 matcher's operands."""
    _need(x, "x", torch.float32, x.device)
    if x.dim() != 2 or x.shape[0] < 1:
        raise ValueError("column_mean takes a matrix with at least one row")
    out = torch.empty((x.shape[1],), dtype=torch.float32, device=x.device)
    check(_lib.lib().spfel_column_mean(_p(x), x.shape[0], x.shape[1], int(bool(round_to_integer)),
                                       _p(out), _stream(x.device)))
    return out


def bf16_centred(x: torch.Tensor, centre: Optional[torch.Tensor] = None) -> tuple:
    """(bf16(x - centre), squared norms of those BF16 rows, upper bounds on
    their rounding-error norms) of a (rows, cols) float32 matrix."""
    _need(x, "x", torch.float32, x.device)
    if x.dim() != 2:
        raise ValueError("bf16_centred takes a matrix")
    if centre is not None:
        _need(centre, "centre", torch.float32, x.device, (x.shape[1],))
    out = torch.empty(tuple(x.shape), dtype=torch.bfloat16, device=x.device)
    n2 = torch.empty((x.shape[0],), dtype=torch.float32, device=x.device)
    err = torch.empty((x.shape[0],), dtype=torch.float32, device=x.device)
    check(_lib.lib().spfel_bf16_centred(_p(x), x.shape[0], x.shape[1], _p(centre), _p(out), _p(n2),
                                        _p(err), _stream(x.device)))
    return out, n2, err


def scale_columns(x: torch.Tensor, g: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x[r][p] * g[p] for a (rows, cols) float32 matrix: with g = sqrt(w),
    matching scaled rows gives the per-pixel weighted distance
    sum_p w_p (s_p - d_p)^2 (a beam stop is w_p = 0)."""
    _need(x, "x", torch.float32, x.device)
    if x.dim() != 2:
        raise ValueError("scale_columns takes a matrix")
    _need(g, "g", torch.float32, x.device, (x.shape[1],))
    if out is None:
        out = torch.empty_like(x)
    else:
        _need(out, "out", torch.float32, x.device, tuple(x.shape))
    check(_lib.lib().spfel_scale_columns(_p(x), x.shape[0], x.shape[1], _p(g), _p(out),
                                         _stream(x.device)))
    return out


def _pixel_scale(pixel_weights, x):
    if pixel_weights is None:
        return None
    w = torch.as_tensor(pixel_weights, dtype=torch.float32, device=x.device)
    if w.shape != (x.shape[1],) or bool((w < 0).any()):
        raise ValueError("pixel_weights must be (P,) and nonnegative")
    return torch.sqrt(w).contiguous()


class ImagesF32:
    """Float32 matcher operand: rows (scaled by sqrt(pixel_weights) when
    given) and their squared norms."""

    def __init__(self, x: torch.Tensor, pixel_weights=None):
        self.g = _pixel_scale(pixel_weights, x)
        self.x = x if self.g is None else scale_columns(x, self.g)
        self.norm2 = row_norm2(self.x)


class ImagesBF16:
    """BF16 matcher operand: the float32 rows (scaled by sqrt(pixel_weights)
    when given), a centre (rounded column mean of those rows unless given),
    and the centred BF16 rows with their norms and rounding-error bounds."""

    def __init__(self, x: torch.Tensor, centre: Optional[torch.Tensor] = None, pixel_weights=None):
        self.g = _pixel_scale(pixel_weights, x)
        self.x = x if self.g is None else scale_columns(x, self.g)
        self.centre = column_mean(self.x) if centre is None else centre
        self.b16, self.norm2, self.err = bf16_centred(self.x, self.centre)


def match_workspace_bytes(M: int, n_img: int, P: int, mode: int = MATCH_FP32) -> int:
    return int(_lib.lib().spfel_match_workspace_bytes(M, n_img, P, mode))


def new_best(n_img: int, device) -> tuple:
    """Initial running best: (best_idx = -1, best_dist = +inf)."""
    return (torch.full((n_img,), -1, dtype=torch.int32, device=device),
            torch.full((n_img,), float("inf"), dtype=torch.float32, device=device))


def _match_operands(slices, slice_norm2, images, image_norm2, best_idx, best_dist, mode,
                    slices_f32, images_f32, slice_err, image_err, flags):
    dt = torch.float32 if mode == MATCH_FP32 else torch.bfloat16
    dev = slices.device
    _need(slices, "slices", dt, dev)
    _need(images, "images", dt, dev)
    if slices.dim() != 2 or images.dim() != 2 or slices.shape[1] != images.shape[1]:
        raise ValueError(f"matcher operands {tuple(slices.shape)} and {tuple(images.shape)}: "
                         "expected (M, P) and (n_img, P)")
    M, P = slices.shape
    n_img = images.shape[0]
    _need(slice_norm2, "slice_norm2", torch.float32, dev, (M,))
    _need(image_norm2, "image_norm2", torch.float32, dev, (n_img,))
    _need(best_idx, "best_idx", torch.int32, dev, (n_img,))
    _need(best_dist, "best_dist", torch.float32, dev, (n_img,))
    if mode != MATCH_FP32:
        _need(slices_f32, "slices_f32", torch.float32, dev, (M, P))
        _need(images_f32, "images_f32", torch.float32, dev, (n_img, P))
        _need(slice_err, "slice_err", torch.float32, dev, (M,))
        _need(image_err, "image_err", torch.float32, dev, (n_img,))
        if flags is not None:
            _need(flags, "flags", torch.int32, dev, (n_img,))
    return dev, M, n_img, P


def match(slices: torch.Tensor, slice_norm2: torch.Tensor, images: torch.Tensor,
          image_norm2: torch.Tensor, best_idx: torch.Tensor, best_dist: torch.Tensor,
          m_offset: int = 0, mode: int = MATCH_FP32, slices_f32: Optional[torch.Tensor] = None,
          images_f32: Optional[torch.Tensor] = None, slice_err: Optional[torch.Tensor] = None,
          image_err: Optional[torch.Tensor] = None, flags: Optional[torch.Tensor] = None,
          workspace: Optional[torch.Tensor] = None) -> tuple:
    """Fold the nearest model image of each image into (best_idx, best_dist)
    in place and return them.  FP32 mode: float32 (M, P) / (n_img, P) rows
    and their norms.  BF16 mode: the outputs of ``bf16_centred`` for both
    sides (one centre), plus the float32 rows and optional per-image
    ``flags`` (int32, |= 1 where the FP32 fallback ran)."""
    dev, M, n_img, P = _match_operands(slices, slice_norm2, images, image_norm2, best_idx,
                                       best_dist, mode, slices_f32, images_f32, slice_err,
                                       image_err, flags)
    need = match_workspace_bytes(M, n_img, P, mode)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty((need,), dtype=torch.uint8, device=dev)
    check(_lib.lib().spfel_match(_p(slices), _p(slice_norm2), _p(images), _p(image_norm2), M,
                                 n_img, P, m_offset, mode, _p(slices_f32), _p(images_f32),
                                 _p(slice_err), _p(image_err), _p(best_idx), _p(best_dist),
                                 _p(flags), _p(workspace), workspace.numel(), _stream(dev)))
    return best_idx, best_dist


def match_noalloc(slices: torch.Tensor, slice_norm2: torch.Tensor, images: torch.Tensor,
                  image_norm2: torch.Tensor, best_idx: torch.Tensor, best_dist: torch.Tensor,
                  m_offset: int = 0, mode: int = MATCH_FP32,
                  slices_f32: Optional[torch.Tensor] = None,
                  images_f32: Optional[torch.Tensor] = None,
                  slice_err: Optional[torch.Tensor] = None,
                  image_err: Optional[torch.Tensor] = None,
                  flags: Optional[torch.Tensor] = None) -> tuple:
    """``match`` through spfel_match_noalloc: the workspace is the library's
    per-device scratch array (nothing is allocated; calls that overlap on
    one GPU race)."""
    dev, M, n_img, P = _match_operands(slices, slice_norm2, images, image_norm2, best_idx,
                                       best_dist, mode, slices_f32, images_f32, slice_err,
                                       image_err, flags)
    with torch.cuda.device(dev):
        check(_lib.lib().spfel_match_noalloc(_p(slices), _p(slice_norm2), _p(images),
                                             _p(image_norm2), M, n_img, P, m_offset, mode,
                                             _p(slices_f32), _p(images_f32), _p(slice_err),
                                             _p(image_err), _p(best_idx), _p(best_dist),
                                             _p(flags), _stream(dev)))
    return best_idx, best_dist


def match_bf16(slices_f32: torch.Tensor, images: "ImagesBF16", best_idx: torch.Tensor,
               best_dist: torch.Tensor, m_offset: int = 0, flags: Optional[torch.Tensor] = None,
               workspace: Optional[torch.Tensor] = None) -> tuple:
    """BF16 matching of float32 model images against prepared images:
    scales the model images' columns as the images' were, centres them with
    the images' centre, then ``match``."""
    s = slices_f32 if images.g is None else scale_columns(slices_f32, images.g)
    sb, sn, se = bf16_centred(s, images.centre)
    return match(sb, sn, images.b16, images.norm2, best_idx, best_dist, m_offset=m_offset,
                 mode=MATCH_BF16_RESCORE8, slices_f32=s, images_f32=images.x,
                 slice_err=se, image_err=images.err, flags=flags, workspace=workspace)


class Normal:
    """Tikhonov-regularised normal equations of Eq. (2) for an N^3 model,
    (A* D A + lambda I) x = A* D b + lambda x0, applied as a convolution with
    the Toeplitz kernel (``set_psf``) and solved by batched conjugate
    gradients, one system per lambda (up to ``max_systems``)."""

    def __init__(self, n_model: int, domain: int = REAL, max_systems: int = 8, device=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.n_model = n_model
        self.domain = domain
        self.max_systems = max_systems
        h = ctypes.c_void_p()
        check(_lib.lib().spfel_normal_create(ctypes.byref(h), n_model, domain, max_systems,
                                             dev.index))
        self._h = h

    @property
    def cdtype(self):
        return torch.complex64 if self.domain == COMPLEX else torch.float32

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value is not None:
            check(_lib.lib().spfel_normal_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_psf(self, psf: torch.Tensor) -> None:
        """Toeplitz kernel on (2N-1)^3 modes: ``merge_adjoint`` of the
        weights on a plan of size 2N-1."""
        M = 2 * self.n_model - 1
        _need(psf, "psf", self.cdtype, self.device, (M, M, M))
        check(_lib.lib().spfel_normal_set_psf(self._h, _p(psf), _stream(self.device)))

    def _lams(self, lambdas):
        lam = [float(v) for v in lambdas]
        if not 1 <= len(lam) <= self.max_systems:
            raise ValueError(f"need 1..{self.max_systems} lambdas, got {len(lam)}")
        return len(lam), (ctypes.c_float * len(lam))(*lam)

    def _vecs(self, x, n, name):
        N = self.n_model
        _need(x, name, self.cdtype, self.device, (n, N, N, N))

    def apply(self, x: torch.Tensor, lambdas) -> torch.Tensor:
        """(A* D A + lambda_s) x[s] for a batch x of shape (n, N, N, N)."""
        n, lam = self._lams(lambdas)
        self._vecs(x, n, "x")
        y = torch.empty_like(x)
        check(_lib.lib().spfel_normal_apply(self._h, _p(x), n, lam, _p(y), _stream(self.device)))
        return y

    def solve(self, rhs: torch.Tensor, x0: torch.Tensor, lambdas, iters: int,
              residuals: bool = False):
        """``iters`` CG steps per lambda from x0; rhs = A* D b.  Returns the
        solutions (n, N, N, N) and, if asked, |r_i| (n, iters + 1)."""
        n, lam = self._lams(lambdas)
        N = self.n_model
        _need(rhs, "rhs", self.cdtype, self.device, (N, N, N))
        _need(x0, "x0", self.cdtype, self.device, (N, N, N))
        x = torch.empty((n, N, N, N), dtype=self.cdtype, device=self.device)
        res = torch.empty((n, iters + 1), dtype=torch.float32, device=self.device) if residuals else None
        check(_lib.lib().spfel_normal_solve(self._h, _p(rhs), _p(x0), n, lam, iters, _p(x),
                                            _p(res), _stream(self.device)))
        return (x, res) if residuals else x

    def lcurve(self, x: torch.Tensor, rhs: torch.Tensor, x0: torch.Tensor, lambdas, bdb: float):
        """(rho, eta) per solution (n, 2) and the L-curve corner index (a
        device int32 scalar)."""
        n, lam = self._lams(lambdas)
        N = self.n_model
        self._vecs(x, n, "x")
        _need(rhs, "rhs", self.cdtype, self.device, (N, N, N))
        _need(x0, "x0", self.cdtype, self.device, (N, N, N))
        re = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        corner = torch.empty((), dtype=torch.int32, device=self.device)
        check(_lib.lib().spfel_normal_lcurve(self._h, _p(x), _p(rhs), _p(x0), n, lam, float(bdb),
                                             _p(re), _p(corner), _stream(self.device)))
        return re, corner


class Phase:
    """Phasing on an N^3 grid (section II-D): ER and HIO iterations between
    the support/positivity constraints and the measured Fourier amplitudes,
    and shrinkwrap support updates."""

    def __init__(self, n: int, device=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.n = n
        h = ctypes.c_void_p()
        check(_lib.lib().spfel_phase_create(ctypes.byref(h), n, dev.index))
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value is not None:
            check(_lib.lib().spfel_phase_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _grid(self, t, name, dtype):
        n = self.n
        _need(t, name, dtype, self.device, (n, n, n))

    def iterate(self, rho: torch.Tensor, amp: torch.Tensor, support: torch.Tensor, n_iter: int,
                mode: int = PHASE_HIO, beta: float = 0.9, positivity: bool = True,
                measured: Optional[torch.Tensor] = None, errors: bool = False):
        """n_iter iterations on rho (N^3 float32) in place; returns the
        per-iteration errors (device float32) if asked."""
        self._grid(rho, "rho", torch.float32)
        self._grid(amp, "amp", torch.float32)
        self._grid(support, "support", torch.uint8)
        if measured is not None:
            self._grid(measured, "measured", torch.uint8)
        err = torch.empty((n_iter,), dtype=torch.float32, device=self.device) if errors else None
        check(_lib.lib().spfel_phase_iterate(self._h, _p(rho), _p(amp), _p(measured), _p(support),
                                             n_iter, mode, float(beta), 1 if positivity else 0,
                                             _p(err), _stream(self.device)))
        return err

    def shrinkwrap(self, rho: torch.Tensor, sigma: float, tau: float,
                   support: Optional[torch.Tensor] = None, blurred: bool = False):
        """New support (N^3 uint8) from the blurred |rho|; with blurred=True
        also returns the blur."""
        self._grid(rho, "rho", torch.float32)
        n = self.n
        if support is None:
            support = torch.empty((n, n, n), dtype=torch.uint8, device=self.device)
        else:
            self._grid(support, "support", torch.uint8)
        b = torch.empty((n, n, n), dtype=torch.float32, device=self.device) if blurred else None
        check(_lib.lib().spfel_phase_shrinkwrap(self._h, _p(rho), float(sigma), float(tau),
                                                _p(support), _p(b), _stream(self.device)))
        return (support, b) if blurred else support
