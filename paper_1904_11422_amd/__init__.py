"""MI355X-native MOFF direct imager (Kent et al. 2019, the EPIC imager).

Python binding of libepic.so: argument marshalling only.  Every step of the
imaging path runs in the library's HIP kernels; PyTorch provides device
memory and streams.  There is no CPU path: the calls raise if the library is
not built or if a tensor is not on the GPU.

    im = Imager(grid_n=64, n_chan=132, n_pol=2, n_ant=256)
    im.set_antennas(xy_m, freq_hz)                     # host float64
    img = im.accumulate(efield, gains)                 # uint8 [T,C,P,A], complex64 [C,P,A]
    g = im.backward(efield, gains, grad_img)           # d loss / d gains
    img = image(im, gains, efield)                     # autograd-aware
    im = Imager(..., remove_autos=True)                # images without the a = b terms
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from ._lib import EpicError, EPIC_FP32, EPIC_SPLIT_FP16, EPIC_SPLIT_BF16  # noqa: F401

_PRECISIONS = {"fp32": EPIC_FP32, "split_fp16": EPIC_SPLIT_FP16, "split_bf16": EPIC_SPLIT_BF16}


def _torch():
    import torch
    return torch


class Imager:
    """One library context: a fixed (N, C, P, A, kernel) configuration."""

    def __init__(self, grid_n: int, n_chan: int, n_pol: int, n_ant: int,
                 kernel_support: int = 3, kernel_sigma_cells: float = 0.5,
                 cell_wavelengths: float = 0.5, precision: str = "fp32",
                 staged: bool = False, timing: bool = False, remove_autos: bool = False,
                 device: Optional[int] = None):
        torch = _torch()
        self.L = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the MOFF imager needs a GPU (no CPU path)")
        self.device = torch.cuda.current_device() if device is None else int(device)
        flags = (_lib.EPIC_FLAG_STAGED if staged else 0) | (_lib.EPIC_FLAG_TIMING if timing else 0) \
            | (_lib.EPIC_FLAG_REMOVE_AUTOS if remove_autos else 0)
        self.cfg = _lib.EpicConfig(grid_n, n_chan, n_pol, n_ant, kernel_support,
                                   kernel_sigma_cells, cell_wavelengths,
                                   _PRECISIONS[precision], flags)
        self.grid_n, self.n_chan, self.n_pol, self.n_ant = grid_n, n_chan, n_pol, n_ant
        self.remove_autos = remove_autos
        self.kernel_support = kernel_support
        self.n_prod = 4 if n_pol == 2 else 1
        ctx = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        st = self.L.epic_init(ctypes.byref(self.cfg), self.device, ctypes.c_void_p(stream),
                              ctypes.byref(ctx))
        _lib.check(self.L, None, st)
        self._ctx = ctx

    # ------------------------------------------------------------------ setup
    def set_antennas(self, xy_m, freq_hz, kernels=None) -> None:
        """Geometry (metres, Hz); kernels: optional complex [C, A, K, K] gridding
        kernels per channel and antenna in place of the Gaussian."""
        xy = np.ascontiguousarray(np.asarray(xy_m, dtype=np.float64))
        f = np.ascontiguousarray(np.asarray(freq_hz, dtype=np.float64))
        if xy.shape != (self.n_ant, 2) or f.shape != (self.n_chan,):
            raise ValueError(f"expected xy_m [{self.n_ant}, 2] and freq_hz [{self.n_chan}]")
        dp = ctypes.POINTER(ctypes.c_double)
        if kernels is None:
            st = self.L.epic_set_antennas(self._ctx, xy.ctypes.data_as(dp), f.ctypes.data_as(dp))
        else:
            K = self.kernel_support
            k = np.ascontiguousarray(np.asarray(kernels, dtype=np.complex64))
            if k.shape != (self.n_chan, self.n_ant, K, K):
                raise ValueError(f"kernels must be [{self.n_chan}, {self.n_ant}, {K}, {K}]")
            st = self.L.epic_set_antennas_kernels(self._ctx, xy.ctypes.data_as(dp),
                                                  f.ctypes.data_as(dp), ctypes.c_void_p(k.ctypes.data))
        _lib.check(self.L, self._ctx, st)

    def _bind_stream(self):
        torch = _torch()
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.L.epic_set_stream(self._ctx, ctypes.c_void_p(s))

    def _check_inputs(self, efield, gains):
        torch = _torch()
        if efield.dtype != torch.uint8 or efield.dim() != 4 or \
                tuple(efield.shape[1:]) != (self.n_chan, self.n_pol, self.n_ant):
            raise ValueError(f"efield must be uint8 [T, {self.n_chan}, {self.n_pol}, {self.n_ant}]")
        if gains.dtype != torch.complex64 or tuple(gains.shape) != (self.n_chan, self.n_pol, self.n_ant):
            raise ValueError(f"gains must be complex64 [{self.n_chan}, {self.n_pol}, {self.n_ant}]")
        for t in (efield, gains):
            if not t.is_cuda or t.device.index != self.device:
                raise ValueError("inputs must be on the imager's GPU")
        return efield.contiguous(), gains.contiguous()

    def image_shape(self):
        return (self.n_chan, self.n_prod, self.grid_n, self.grid_n)

    # ------------------------------------------------------------------ calls
    def accumulate(self, efield, gains, image=None, reset: bool = True):
        """Sum of polarised images over the samples of efield (complex128);
        with remove_autos=True, less the antenna autocorrelations of these samples."""
        torch = _torch()
        efield, gains = self._check_inputs(efield, gains)
        if image is None:
            image = torch.empty(self.image_shape(), dtype=torch.complex128,
                                device=efield.device)
        elif image.dtype != torch.complex128 or tuple(image.shape) != self.image_shape() or \
                not image.is_contiguous() or not image.is_cuda:
            raise ValueError("image must be a contiguous complex128 CUDA tensor "
                             f"{self.image_shape()}")
        self._bind_stream()
        st = self.L.epic_image_accumulate(self._ctx, ctypes.c_void_p(efield.data_ptr()),
                                          int(efield.shape[0]), ctypes.c_void_p(gains.data_ptr()),
                                          ctypes.c_void_p(image.data_ptr()), 1 if reset else 0)
        _lib.check(self.L, self._ctx, st)
        return image

    def accumulate_noalloc(self, efield, gains, image, reset: bool = True):
        """accumulate() through epic_image_accumulate_noalloc: the caller passes
        the image, and the library's partial slots are its static scratch
        array, so the call allocates nothing (fused float32 kernels only)."""
        torch = _torch()
        efield, gains = self._check_inputs(efield, gains)
        if image.dtype != torch.complex128 or tuple(image.shape) != self.image_shape() or \
                not image.is_contiguous() or not image.is_cuda:
            raise ValueError("image must be a contiguous complex128 CUDA tensor "
                             f"{self.image_shape()}")
        self._bind_stream()
        st = self.L.epic_image_accumulate_noalloc(self._ctx, ctypes.c_void_p(efield.data_ptr()),
                                                  int(efield.shape[0]),
                                                  ctypes.c_void_p(gains.data_ptr()),
                                                  ctypes.c_void_p(image.data_ptr()), 1 if reset else 0)
        _lib.check(self.L, self._ctx, st)
        return image

    def postprocess(self, image, taper_floor: Optional[float] = None, out=None):
        """Pseudo-Stokes planes I, Q, U, V (XX for one polarisation), float64
        [C, 4 or 1, N, N]; with taper_floor (0..1) divided by the kernel taper
        where it is at least taper_floor times the channel's maximum."""
        torch = _torch()
        if image.dtype != torch.complex128 or tuple(image.shape) != self.image_shape() or \
                not image.is_contiguous() or not image.is_cuda:
            raise ValueError(f"image must be a contiguous CUDA complex128 tensor {self.image_shape()}")
        shape = (self.n_chan, self.n_prod, self.grid_n, self.grid_n)
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=image.device)
        elif tuple(out.shape) != shape or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float64 tensor {shape}")
        self._bind_stream()
        st = self.L.epic_postprocess(self._ctx, ctypes.c_void_p(image.data_ptr()),
                                     -1.0 if taper_floor is None else float(taper_floor),
                                     ctypes.c_void_p(out.data_ptr()))
        _lib.check(self.L, self._ctx, st)
        return out

    def kernel_taper(self):
        """The kernel taper of the current geometry, float64 [C, N, N] (fftshifted)."""
        torch = _torch()
        out = torch.empty((self.n_chan, self.grid_n, self.grid_n), dtype=torch.float64,
                          device=f"cuda:{self.device}")
        self._bind_stream()
        _lib.check(self.L, self._ctx, self.L.epic_kernel_taper(self._ctx, ctypes.c_void_p(out.data_ptr())))
        return out

    def frontend(self, raw, c0: int = 0, c_step: int = 1, out=None):
        """Decimate and transpose a gulp in arrival order, uint8 [T, c_in, A, P]
        on the GPU, into the imaging layout [T, C, P, A] (channel i = c0 + i c_step)."""
        torch = _torch()
        if raw.dtype != torch.uint8 or raw.dim() != 4 or \
                tuple(raw.shape[2:]) != (self.n_ant, self.n_pol) or not raw.is_cuda:
            raise ValueError(f"raw must be a CUDA uint8 tensor [T, c_in, {self.n_ant}, {self.n_pol}]")
        raw = raw.contiguous()
        shape = (raw.shape[0], self.n_chan, self.n_pol, self.n_ant)
        if out is None:
            out = torch.empty(shape, dtype=torch.uint8, device=raw.device)
        elif tuple(out.shape) != shape or out.dtype != torch.uint8 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous uint8 tensor {shape}")
        self._bind_stream()
        st = self.L.epic_frontend(self._ctx, ctypes.c_void_p(raw.data_ptr()), int(raw.shape[0]),
                                  int(raw.shape[1]), int(c0), int(c_step),
                                  ctypes.c_void_p(out.data_ptr()))
        _lib.check(self.L, self._ctx, st)
        return out

    def backward(self, efield, gains, grad_image):
        """d loss / d gains (dL/dRe + i dL/dIm, complex64 [C, P, A])."""
        torch = _torch()
        efield, gains = self._check_inputs(efield, gains)
        grad_image = grad_image.to(torch.complex128).contiguous()
        if tuple(grad_image.shape) != self.image_shape():
            raise ValueError(f"grad_image must be {self.image_shape()}")
        out = torch.empty((self.n_chan, self.n_pol, self.n_ant), dtype=torch.complex64,
                          device=efield.device)
        self._bind_stream()
        st = self.L.epic_image_backward(self._ctx, ctypes.c_void_p(efield.data_ptr()),
                                        int(efield.shape[0]), ctypes.c_void_p(gains.data_ptr()),
                                        ctypes.c_void_p(grad_image.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()))
        _lib.check(self.L, self._ctx, st)
        return out

    def last_timing(self):
        """(main kernel ms, whole call ms) of the last call (timing=True)."""
        m, c = ctypes.c_float(), ctypes.c_float()
        st = self.L.epic_last_timing(self._ctx, ctypes.byref(m), ctypes.byref(c))
        _lib.check(self.L, self._ctx, st)
        return m.value, c.value

    def timing_history(self, n):
        """Main-kernel ms of the last n timed calls, oldest first (timing=True);
        waits only for the last of them."""
        buf = (ctypes.c_float * int(n))()
        _lib.check(self.L, self._ctx, self.L.epic_timing_history(self._ctx, int(n), buf))
        return list(buf)

    def last_autos_timing(self):
        """(autocorrelation-sum kernel ms, whole removal ms) of the last call
        (timing=True, remove_autos=True)."""
        m, r = ctypes.c_float(), ctypes.c_float()
        st = self.L.epic_last_autos_timing(self._ctx, ctypes.byref(m), ctypes.byref(r))
        _lib.check(self.L, self._ctx, st)
        return m.value, r.value

    def last_kernel_name(self) -> str:
        return self.L.epic_last_kernel_name(self._ctx).decode()

    def close(self):
        if getattr(self, "_ctx", None):
            self.L.epic_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pipeline:
    """Double-buffered streaming of gulps from pinned host memory into an
    Imager: copy of gulp i overlaps the front end and imaging of gulp i - 1."""

    def __init__(self, imager: Imager, n_time: int, c_in: int, c0: int = 0, c_step: int = 1,
                 sample_s: float = 40e-6):
        self.imager, self.L = imager, imager.L
        self.n_time, self.c_in = int(n_time), int(c_in)
        imager._bind_stream()
        p = ctypes.c_void_p()
        st = self.L.epic_pipeline_create(imager._ctx, self.n_time, self.c_in, int(c0), int(c_step),
                                         float(sample_s), ctypes.byref(p))
        _lib.check_pipeline(self.L, None, st)
        self._p = p
        self._held = []          # host gulps whose copies may still be pending

    def push(self, host_raw, gains, image, reset: bool = True):
        """host_raw: CPU uint8 [n_time, c_in, A, P] (pinned for overlap); gains and
        image on the GPU as for Imager.accumulate."""
        torch = _torch()
        im = self.imager
        if host_raw.dtype != torch.uint8 or host_raw.is_cuda or not host_raw.is_contiguous() or \
                tuple(host_raw.shape) != (self.n_time, self.c_in, im.n_ant, im.n_pol):
            raise ValueError("host_raw must be a contiguous CPU uint8 tensor "
                             f"[{self.n_time}, {self.c_in}, {im.n_ant}, {im.n_pol}]")
        if gains.dtype != torch.complex64 or tuple(gains.shape) != (im.n_chan, im.n_pol, im.n_ant) \
                or not gains.is_cuda:
            raise ValueError("gains must be a CUDA complex64 tensor [C, P, A]")
        if image.dtype != torch.complex128 or tuple(image.shape) != im.image_shape() or \
                not image.is_contiguous() or not image.is_cuda:
            raise ValueError(f"image must be a contiguous CUDA complex128 tensor {im.image_shape()}")
        gains = gains.contiguous()
        self._held.append((host_raw, gains))
        if len(self._held) > 2 * 64:
            self._held = self._held[-64:]        # the library waits for older gulps
        st = self.L.epic_pipeline_push(self._p, ctypes.c_void_p(host_raw.data_ptr()),
                                       ctypes.c_void_p(gains.data_ptr()),
                                       ctypes.c_void_p(image.data_ptr()), 1 if reset else 0)
        _lib.check_pipeline(self.L, self._p, st)

    def report(self) -> dict:
        """Wait for every pushed gulp; statistics (ms) and the real-time check."""
        s = _lib.PipelineStats()
        _lib.check_pipeline(self.L, self._p, self.L.epic_pipeline_report(self._p, ctypes.byref(s)))
        self._held = []
        return {k: getattr(s, k) for k, _ in _lib.PipelineStats._fields_}

    def close(self):
        if getattr(self, "_p", None):
            self.L.epic_pipeline_destroy(self._p)
            self._p = None
            self._held = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_image_fn():
    torch = _torch()

    class ImageFn(torch.autograd.Function):
        """image = accumulate(efield, gains); backward gives d loss / d gains."""

        @staticmethod
        def forward(ctx, gains, efield, imager):
            ctx.imager = imager
            ctx.save_for_backward(gains, efield)
            return imager.accumulate(efield, gains.contiguous())

        @staticmethod
        def backward(ctx, grad_image):
            gains, efield = ctx.saved_tensors
            g = ctx.imager.backward(efield, gains.contiguous(), grad_image)
            return g, None, None

    return ImageFn


_IMAGE_FN = None


def image(imager: Imager, gains, efield):
    """Autograd-aware accumulated image (gains may be an expanded view)."""
    global _IMAGE_FN
    if _IMAGE_FN is None:
        _IMAGE_FN = _make_image_fn()
    return _IMAGE_FN.apply(gains, efield, imager)


class Batch:
    """Several imaging configurations advanced together (one context and
    stream per block, fork-join on the caller's stream), with optional HIP
    graph capture/replay and an autotuned launch shape per block."""

    def __init__(self, configs, device: Optional[int] = None):
        """configs: list of dicts with the Imager keyword arguments."""
        torch = _torch()
        self.L = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the MOFF imager needs a GPU (no CPU path)")
        self.device = torch.cuda.current_device() if device is None else int(device)
        arr = (_lib.EpicConfig * len(configs))()
        self.shapes = []
        for i, c in enumerate(configs):
            arr[i] = _lib.EpicConfig(c["grid_n"], c["n_chan"], c["n_pol"], c["n_ant"],
                                     c.get("kernel_support", 3), c.get("kernel_sigma_cells", 0.5),
                                     c.get("cell_wavelengths", 0.5),
                                     _PRECISIONS[c.get("precision", "fp32")],
                                     (_lib.EPIC_FLAG_STAGED if c.get("staged") else 0)
                                     | (_lib.EPIC_FLAG_REMOVE_AUTOS if c.get("remove_autos") else 0))
            self.shapes.append((c["n_chan"], 4 if c["n_pol"] == 2 else 1, c["grid_n"], c["grid_n"]))
        self.n_blocks = len(configs)
        b = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        st = self.L.epic_batch_create(arr, len(configs), self.device, ctypes.c_void_p(stream),
                                      ctypes.byref(b))
        _lib.check_batch(self.L, None, st)
        self._b = b

    def set_antennas(self, block: int, xy_m, freq_hz):
        xy = np.ascontiguousarray(np.asarray(xy_m, dtype=np.float64))
        f = np.ascontiguousarray(np.asarray(freq_hz, dtype=np.float64))
        dp = ctypes.POINTER(ctypes.c_double)
        st = self.L.epic_batch_set_antennas(self._b, block, xy.ctypes.data_as(dp), f.ctypes.data_as(dp))
        _lib.check_batch(self.L, self._b, st)

    def _ptrs(self, tensors):
        if len(tensors) != self.n_blocks:
            raise ValueError(f"expected {self.n_blocks} tensors")
        for t in tensors:
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("batch tensors must be contiguous CUDA tensors")
        return (ctypes.c_void_p * self.n_blocks)(*[t.data_ptr() for t in tensors])

    def new_images(self):
        torch = _torch()
        return [torch.empty(s, dtype=torch.complex128, device=f"cuda:{self.device}")
                for s in self.shapes]

    def _args(self, efields, gains, images):
        n_time = int(efields[0].shape[0])
        if any(int(e.shape[0]) != n_time for e in efields):
            raise ValueError("all blocks must have the same number of samples")
        return self._ptrs(efields), n_time, self._ptrs(gains), self._ptrs(images)

    def accumulate(self, efields, gains, images, reset: bool = True):
        e, n, g, im = self._args(efields, gains, images)
        st = self.L.epic_batch_accumulate(self._b, e, n, g, im, 1 if reset else 0)
        _lib.check_batch(self.L, self._b, st)
        return images

    def capture(self, efields, gains, images, reset: bool = True):
        self._keep = (efields, gains, images)          # the graph reads these buffers
        e, n, g, im = self._args(efields, gains, images)
        st = self.L.epic_batch_capture(self._b, e, n, g, im, 1 if reset else 0)
        _lib.check_batch(self.L, self._b, st)

    def replay(self):
        _lib.check_batch(self.L, self._b, self.L.epic_batch_replay(self._b))

    def tune(self, efields, gains, images, cache_path: Optional[str] = None) -> bool:
        e, n, g, im = self._args(efields, gains, images)
        measured = ctypes.c_int32()
        path = cache_path.encode() if cache_path else None
        st = self.L.epic_batch_tune(self._b, e, n, g, im, path, ctypes.byref(measured))
        _lib.check_batch(self.L, self._b, st)
        return bool(measured.value)

    def plan(self):
        out = []
        for i in range(self.n_blocks):
            gsz, tb = ctypes.c_int32(), ctypes.c_int32()
            self.L.epic_batch_plan(self._b, i, ctypes.byref(gsz), ctypes.byref(tb))
            out.append((gsz.value, tb.value))
        return out

    def set_launch(self, launch: int, grid: int, team: int = 0, kblock: int = 128, xcd: bool = True):
        """Shape of grouped launch `launch` by hand (grid 0: the resident
        maximum; team 0: chosen from the number of samples)."""
        _lib.check_batch(self.L, self._b, self.L.epic_batch_set_launch(self._b, int(launch), int(grid),
                                                                       int(team), int(kblock),
                                                                       1 if xcd else 0))

    def launch_plan(self):
        """Per block: (launch index, blocks that launch walks -- 0 when the
        block runs alone through its context --, team size, float32 block
        length, XCD order flag)."""
        out = []
        for i in range(self.n_blocks):
            v = [ctypes.c_int32() for _ in range(5)]
            _lib.check_batch(self.L, self._b,
                             self.L.epic_batch_launch_plan(self._b, i, *[ctypes.byref(x) for x in v]))
            out.append(tuple(x.value for x in v))
        return out

    @property
    def serial(self) -> bool:
        """True if the launches run one after another (the tuner's choice)."""
        return bool(self.L.epic_batch_serial(self._b))

    @serial.setter
    def serial(self, value: bool):
        _lib.check_batch(self.L, self._b, self.L.epic_batch_set_serial(self._b, 1 if value else 0))

    def close(self):
        if getattr(self, "_b", None):
            self.L.epic_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
