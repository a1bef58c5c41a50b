"""Python binding of libhfx (plane-wave Gamma-point exact exchange on gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libhfx.so``.  PyTorch supplies device memory and the current
stream.  The C entry points are described in ``include/hfx.h``; the Python
names are the same without the ``hfx_`` prefix.

Conventions (Methods, MTACE subsection: Eqs. vx, vij, HFX and the ACE matrix M):
``kpsi`` = V_X psi, ``ex`` = 1/2 sum_i <psi_i|K psi_i> (half the paper's
closed-shell Eq. HFX), ``m[k, l]`` = <psi_k|K psi_l>, dE_x/dpsi = 2 dV K psi.
Orbitals are float64 tensors ``[n_orb, n, n, n]`` (z, y, x) on the GPU.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfx.so")

TRUNCATED = 0
ERFC = 1
FP32 = 0
FP64 = 1
ORTHO_LOWDIN = 0
ORTHO_CHOLESKY = 1
GRAPH_ENERGY = 0
GRAPH_APPLY = 1
GRAPH_STEP = 2
PASSES = ("stage", "zero", "pair_fwd", "plane", "rows_fwd", "cols_conv", "rows_inv", "inv_acc",
          "inv_energy", "energy_reduce", "contract", "ortho", "scale", "ace_build", "ace_apply",
          "scdm")

_STATUS = {0: "HFX_OK", 1: "HFX_EINVAL", 2: "HFX_EUNSUPPORTED", 3: "HFX_ENOMEM",
           4: "HFX_EDEVICE"}


def variants(n, precision=FP32):
    """Names of the compiled kernel configurations for an n^3 grid (default first)."""
    v = load_library().hfx_variants(int(n), int(precision)).decode()
    return [x for x in v.split(";") if x]


class HfxError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__(f"{_STATUS.get(status, status)}: {detail}")


class System(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("L", ctypes.c_double * 3), ("n_orb", ctypes.c_int),
                ("kernel", ctypes.c_int), ("param", ctypes.c_double)]


_lib = None


def load_library(path=None):
    """Load libhfx.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not found: build it with `python -m paper_2309_00651_amd.build`")
    lib = ctypes.CDLL(p)
    vp, i, sz, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
    lib.hfx_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(System), i, i,
                                    ctypes.c_char_p]
    lib.hfx_plan_destroy.argtypes = [vp]
    lib.hfx_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.hfx_exchange_energy.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.hfx_apply_exchange.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.hfx_exchange_matrix.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.hfx_exchange_matrix_kpsi.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.hfx_orthonormalize.argtypes = [vp, vp, i, vp, sz, vp]
    lib.hfx_exchange_gradient.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.hfx_profile_enable.argtypes = [vp, i]
    lib.hfx_profile_read.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(d),
                                     ctypes.POINTER(ctypes.c_longlong), i]
    lib.hfx_ace_build.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.hfx_ace_apply.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.hfx_screen.argtypes = [vp, vp, d, ctypes.POINTER(ctypes.c_longlong), vp, sz, vp]
    lib.hfx_scdm.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.hfx_schedule_info.argtypes = [vp, i, ctypes.POINTER(ctypes.c_longlong)]
    lib.hfx_plan_describe.argtypes = [vp, i]
    lib.hfx_plan_describe.restype = ctypes.c_char_p
    lib.hfx_autotune.argtypes = [ctypes.POINTER(System), i, i, ctypes.c_char_p, vp, i,
                                 ctypes.c_char_p, ctypes.c_char_p, sz, vp]
    lib.hfx_graph_create.argtypes = [vp, i, vp, vp, vp, vp, vp, sz, ctypes.POINTER(vp)]
    lib.hfx_graph_launch.argtypes = [vp, vp]
    lib.hfx_graph_destroy.argtypes = [vp]
    lib.hfx_variants.argtypes = [i, i]
    lib.hfx_variants.restype = ctypes.c_char_p
    lib.hfx_status_string.argtypes = [i]
    lib.hfx_status_string.restype = ctypes.c_char_p
    lib.hfx_last_error.argtypes = []
    lib.hfx_last_error.restype = ctypes.c_char_p
    for name in ("hfx_plan_create", "hfx_plan_destroy", "hfx_workspace_size",
                 "hfx_exchange_energy", "hfx_apply_exchange", "hfx_exchange_matrix",
                 "hfx_exchange_matrix_kpsi", "hfx_orthonormalize", "hfx_exchange_gradient", "hfx_profile_enable",
                 "hfx_profile_read", "hfx_graph_create", "hfx_graph_launch",
                 "hfx_graph_destroy", "hfx_ace_build", "hfx_ace_apply", "hfx_screen", "hfx_scdm",
                 "hfx_schedule_info", "hfx_autotune"):
        getattr(lib, name).restype = i
    if path is None:
        _lib = lib
    return lib


def _check(status):
    if status != 0:
        raise HfxError(status, _lib.hfx_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass(frozen=True)
class SystemSpec:
    n: object          # grid points per axis (cubic), or (nx, ny, nz) with nx == ny
    box: tuple
    n_orb: int
    kernel: int = TRUNCATED
    param: float = 0.0

    @property
    def shape_xyz(self):
        return tuple(int(x) for x in self.n) if isinstance(self.n, (tuple, list)) \
            else (int(self.n),) * 3

    def to_c(self):
        s = System()
        for k, v in enumerate(self.shape_xyz):
            s.n[k] = v
        for k in range(3):
            s.L[k] = float(self.box[k])
        s.n_orb = int(self.n_orb)
        s.kernel = int(self.kernel)
        s.param = float(self.param)
        return s

    @property
    def nr(self):
        nx, ny, nz = self.shape_xyz
        return nx * ny * nz

    @property
    def dv(self):
        return self.box[0] * self.box[1] * self.box[2] / self.nr


class Plan:
    """A libhfx plan for one or more systems (concatenated in plan order)."""

    def __init__(self, systems, precision=FP32, options=None, device=None):
        lib = load_library()
        if isinstance(systems, SystemSpec):
            systems = [systems]
        self.systems = list(systems)
        self.precision = precision
        self.device = torch.device(device or "cuda")
        arr = (System * len(self.systems))(*[s.to_c() for s in self.systems])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.hfx_plan_create(ctypes.byref(h), arr, len(self.systems), int(precision),
                                       options.encode() if options else None))
        self._h = h
        nbytes = ctypes.c_size_t()
        _check(lib.hfx_workspace_size(self._h, ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        self._ws = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(_lib.hfx_plan_destroy(self._h))
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers -----------------------------------------------------------
    def workspace(self):
        if self._ws is None or self._ws.numel() < self.ws_bytes:
            self._ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=self.device)
        return self._ws

    @property
    def total_orb_points(self):
        return sum(s.n_orb * s.nr for s in self.systems)

    @property
    def kpsi_dtype(self):
        return torch.float32 if self.precision == FP32 else torch.float64

    def _check_psi(self, psi):
        if psi.dtype != torch.float64 or not psi.is_cuda or not psi.is_contiguous():
            raise ValueError("psi must be a contiguous float64 CUDA tensor")
        if psi.numel() != self.total_orb_points:
            raise ValueError(f"psi has {psi.numel()} values, plan expects {self.total_orb_points}")

    # -- entry points ------------------------------------------------------
    def exchange_energy(self, psi, ex=None):
        self._check_psi(psi)
        if ex is None:
            ex = torch.empty(len(self.systems), dtype=torch.float64, device=self.device)
        ws = self.workspace()
        _check(_lib.hfx_exchange_energy(self._h, _ptr(psi), _ptr(ex), _ptr(ws), self.ws_bytes,
                                        _stream()))
        return ex

    def apply_exchange(self, psi, kpsi=None, ex=None, with_energy=True):
        self._check_psi(psi)
        if kpsi is None:
            kpsi = torch.empty(psi.shape, dtype=self.kpsi_dtype, device=self.device)
        if with_energy and ex is None:
            ex = torch.empty(len(self.systems), dtype=torch.float64, device=self.device)
        ws = self.workspace()
        _check(_lib.hfx_apply_exchange(self._h, _ptr(psi), _ptr(kpsi),
                                       _ptr(ex) if with_energy else ctypes.c_void_p(0),
                                       _ptr(ws), self.ws_bytes, _stream()))
        return kpsi, ex

    def exchange_matrix(self, psi, kpsi=None, m=None, ex=None):
        """M = dV Psi^T (K Psi) (float64, systems' n_orb^2 blocks concatenated).

        Without ``kpsi`` the library forms K psi itself (hfx_exchange_matrix,
        which also writes E_x into ``ex`` when given); with ``kpsi`` (from
        apply_exchange of this plan) only the contraction runs
        (hfx_exchange_matrix_kpsi)."""
        self._check_psi(psi)
        if m is None:
            m = torch.empty(sum(s.n_orb ** 2 for s in self.systems), dtype=torch.float64,
                            device=self.device)
        ws = self.workspace()
        if kpsi is None:
            _check(_lib.hfx_exchange_matrix(self._h, _ptr(psi), _ptr(m), _ptr(ex), _ptr(ws),
                                            self.ws_bytes, _stream()))
            return m
        if kpsi.dtype != self.kpsi_dtype or kpsi.numel() != psi.numel():
            raise ValueError("kpsi must come from apply_exchange of this plan")
        _check(_lib.hfx_exchange_matrix_kpsi(self._h, _ptr(psi), _ptr(kpsi), _ptr(m), _ptr(ws),
                                             self.ws_bytes, _stream()))
        return m

    def exchange_gradient(self, psi, gscale=None, grad=None):
        """dE_x/dpsi = 2 dV gscale K psi (float64), pair potentials recomputed."""
        self._check_psi(psi)
        if grad is None:
            grad = torch.empty(psi.shape, dtype=torch.float64, device=self.device)
        if gscale is not None:
            gscale = gscale.to(device=self.device, dtype=torch.float64).contiguous()
        ws = self.workspace()
        _check(_lib.hfx_exchange_gradient(self._h, _ptr(psi), _ptr(gscale), _ptr(grad),
                                          _ptr(ws), self.ws_bytes, _stream()))
        return grad

    def orthonormalize(self, psi, method=ORTHO_LOWDIN):
        self._check_psi(psi)
        ws = self.workspace()
        _check(_lib.hfx_orthonormalize(self._h, _ptr(psi), int(method), _ptr(ws), self.ws_bytes,
                                       _stream()))
        return psi

    def ace_build(self, kpsi, m, p=None):
        """ACE projectors P = W L^(-T) (rows |P_k>, float64, the layout of psi)
        from W = K psi (apply_exchange) and M (exchange_matrix)."""
        if kpsi.dtype != self.kpsi_dtype or kpsi.numel() != self.total_orb_points:
            raise ValueError("kpsi must come from apply_exchange of this plan")
        if m.dtype != torch.float64 or m.numel() != sum(s.n_orb ** 2 for s in self.systems):
            raise ValueError("m must come from exchange_matrix of this plan")
        if p is None:
            p = torch.empty(kpsi.shape, dtype=torch.float64, device=self.device)
        self._check_psi(p)
        ws = self.workspace()
        _check(_lib.hfx_ace_build(self._h, _ptr(kpsi), _ptr(m), _ptr(p), _ptr(ws), self.ws_bytes,
                                  _stream()))
        return p

    def ace_apply(self, p, phi, out=None):
        """out = V_X^ACE phi = -sum_k P_k <P_k|phi>, row by row (float64)."""
        self._check_psi(p)
        self._check_psi(phi)
        if out is None:
            out = torch.empty(phi.shape, dtype=torch.float64, device=self.device)
        self._check_psi(out)
        ws = self.workspace()
        _check(_lib.hfx_ace_apply(self._h, _ptr(p), _ptr(phi), _ptr(out), _ptr(ws), self.ws_bytes,
                                  _stream()))
        return out

    def screen(self, psi, rho_cut):
        """s-MTACE pair screening: later calls sum over the pairs with
        int |psi_a psi_b| >= rho_cut only (rho_cut <= 0: all pairs again).
        Returns the number of kept pairs a <= b of each system."""
        self._check_psi(psi)
        kept = (ctypes.c_longlong * len(self.systems))()
        ws = self.workspace()
        _check(_lib.hfx_screen(self._h, _ptr(psi), float(rho_cut), kept, _ptr(ws), self.ws_bytes,
                               _stream()))
        return list(kept)

    def scdm(self, psi, phi=None, pivots=None):
        """SCDM-localised orthonormal orbitals of psi (float64, the layout of
        psi; phi may be psi itself) and the selected grid points (int32, one
        per orbital, flat index (z n + y) n + x)."""
        self._check_psi(psi)
        if phi is None:
            phi = torch.empty_like(psi)
        self._check_psi(phi)
        if pivots is None:
            pivots = torch.empty(sum(s.n_orb for s in self.systems), dtype=torch.int32,
                                 device=self.device)
        ws = self.workspace()
        _check(_lib.hfx_scdm(self._h, _ptr(psi), _ptr(phi), _ptr(pivots), _ptr(ws),
                             self.ws_bytes, _stream()))
        return phi, pivots

    def schedule_info(self, system=0):
        """(batches, tile pairs, pair grids, orbital pairs) of the current schedule."""
        info = (ctypes.c_longlong * 4)()
        _check(_lib.hfx_schedule_info(self._h, int(system), info))
        return tuple(info)

    def describe(self, system=0):
        """Kernel configuration and schedule of one system, as one line."""
        d = _lib.hfx_plan_describe(self._h, int(system))
        if d is None:
            raise HfxError(1, _lib.hfx_last_error().decode())
        return d.decode()

    def graph(self, op, psi, kpsi=None, ex=None, m=None):
        """Capture one call (GRAPH_ENERGY / GRAPH_APPLY / GRAPH_STEP) for these buffers."""
        self._check_psi(psi)
        ws = self.workspace()
        h = ctypes.c_void_p()
        _check(_lib.hfx_graph_create(self._h, int(op), _ptr(psi), _ptr(kpsi), _ptr(ex), _ptr(m),
                                     _ptr(ws), self.ws_bytes, ctypes.byref(h)))
        return Graph(h, self, (psi, kpsi, ex, m, ws))

    def profile(self, enable=True):
        _check(_lib.hfx_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """{pass: dict(ms, bytes, flops, launches)} since the last read (waits for events)."""
        n = len(PASSES)
        ms, by, fl = (ctypes.c_double * n)(), (ctypes.c_double * n)(), (ctypes.c_double * n)()
        la = (ctypes.c_longlong * n)()
        _check(_lib.hfx_profile_read(self._h, ms, by, fl, la, n))
        return {PASSES[k]: dict(ms=ms[k], bytes=by[k], flops=fl[k], launches=la[k])
                for k in range(n) if la[k]}

    def split(self, flat):
        """Views of a concatenated per-system buffer (orbital-shaped)."""
        out, off = [], 0
        for s in self.systems:
            k = s.n_orb * s.nr
            nx, ny, nz = s.shape_xyz
            out.append(flat.reshape(-1)[off:off + k].view(s.n_orb, nz, ny, nx))
            off += k
        return out


class Graph:
    """A captured libhfx call; launch() replays it on the current stream."""

    def __init__(self, handle, plan, keep):
        self._h = handle
        self.plan = plan          # the plan must outlive the graph
        self._keep = keep         # buffers baked into the graph

    def launch(self):
        _check(_lib.hfx_graph_launch(self._h, _stream()))

    def close(self):
        if self._h is not None and self._h.value:
            _check(_lib.hfx_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_plans = {}


def _plan_for(psi, box, kernel, param, precision):
    n = psi.shape[-1]
    key = (n, tuple(float(b) for b in box), psi.shape[0], kernel, float(param), precision,
           psi.device)
    p = _plans.get(key)
    if p is None:
        p = Plan(SystemSpec(n, tuple(box), psi.shape[0], kernel, param), precision,
                 device=psi.device)
        _plans[key] = p
    return p


def exchange_energy(psi, box, kernel=TRUNCATED, param=0.0, precision=FP32):
    """E_x of one system (float64 scalar tensor on the GPU)."""
    return _plan_for(psi, box, kernel, param, precision).exchange_energy(psi)[0]


def apply_exchange(psi, box, kernel=TRUNCATED, param=0.0, precision=FP32):
    """(K psi, E_x) of one system."""
    kpsi, ex = _plan_for(psi, box, kernel, param, precision).apply_exchange(psi)
    return kpsi, ex[0]


def exchange_matrix(psi, box, kernel=TRUNCATED, param=0.0, precision=FP32):
    """(M, K psi, E_x) of one system; M = dV Psi^T (K Psi)."""
    p = _plan_for(psi, box, kernel, param, precision)
    kpsi, ex = p.apply_exchange(psi)
    m = p.exchange_matrix(psi, kpsi)
    return m.view(psi.shape[0], psi.shape[0]), kpsi, ex[0]


def orthonormalize(psi, box, precision=FP64):
    """In-place Loewdin orthonormalisation (float64 on the GPU)."""
    return _plan_for(psi, box, TRUNCATED, 0.0, precision).orthonormalize(psi)


class ExchangeEnergy(torch.autograd.Function):
    """E_x(Psi) with the K psi kernel as its backward: dE_x/dpsi = 2 dV K psi.

    The forward stores only Psi; the backward recomputes the pair potentials
    through ``apply_exchange`` instead of keeping them.
    """

    @staticmethod
    def forward(ctx, psi, plan):
        ex = plan.exchange_energy(psi.contiguous())
        ctx.save_for_backward(psi)
        ctx.plan = plan
        return ex

    @staticmethod
    def backward(ctx, grad_ex):
        (psi,) = ctx.saved_tensors
        grad = ctx.plan.exchange_gradient(psi.contiguous(), gscale=grad_ex)
        return grad, None


def exchange_energy_autograd(psi, plan):
    return ExchangeEnergy.apply(psi, plan)
