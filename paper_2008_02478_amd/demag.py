"""PyTorch front end of the demagnetizing-field library.

PyTorch supplies device memory and the current stream; the arithmetic runs
in the library (include/demag.h).  A DemagPlan owns the plan and the two
device buffers it needs.
"""
import ctypes
import math

import torch

from . import lib as _l

MU0 = 4e-7 * math.pi


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class _Schedules:
    """Launch schedules of a plan's parts (see demag_set_schedule)."""

    def schedules(self):
        """[{"yg", "kw", "radix"}, ...], one dict per part."""
        n = ctypes.c_int()
        _l.check(self._lib.demag_schedule_count(self._p, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            yg, kw, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            _l.check(self._lib.demag_get_schedule(self._p, i, ctypes.byref(yg), ctypes.byref(kw), ctypes.byref(r)))
            out.append({"yg": yg.value, "kw": kw.value, "radix": r.value})
        return out

    def set_schedule(self, part, yg=0, kw=0, radix=0):
        _l.check(self._lib.demag_set_schedule(self._p, int(part), int(yg), int(kw), int(radix)))

    def z_passes(self, part=0):
        """True when the part transforms along z in separate passes."""
        v = ctypes.c_int()
        _l.check(self._lib.demag_get_z_passes(self._p, int(part), ctypes.byref(v)))
        return bool(v.value)

    def set_z_passes(self, separate, part=0):
        _l.check(self._lib.demag_set_z_passes(self._p, int(part), int(bool(separate))))

    def autotune(self, cache=None, force=False, keep_form=False):
        """Pick each part's launch schedule by timing the candidates on the
        current stream (or from the JSON cache file `cache`, which is updated
        with what was measured).  keep_form: keep the current z form (fused
        or separate passes).  Returns the number of parts measured."""
        with torch.cuda.device(self.device):
            m = torch.zeros(self._vec_shape, dtype=torch.float32, device=self.device)
            H = torch.empty_like(m)
            n = ctypes.c_int()
            path = None if cache is None else str(cache).encode()
            flags = (_l.TUNE_FORCE if force else 0) | (_l.TUNE_KEEP_FORM if keep_form else 0)
            _l.check(self._lib.demag_autotune(self._p, _ptr(m), _ptr(H), path, flags,
                                              ctypes.byref(n), _stream()))
        return n.value


class DemagPlan(_Schedules):
    """Plan for one mesh of n = (nx, ny, nz) cells of size cell = (dx, dy, dz)
    metres.  pbc: OR of lib.PBC_X / PBC_Y / PBC_Z for periodic axes (multiple
    images, `images` on either side; 0 = the library default).  Builds the
    kernel spectrum on construction."""

    def __init__(self, n, cell, device=None, pbc=0, images=0):
        self._lib = _l.load()
        self.n = tuple(int(v) for v in n)
        self.cell = tuple(float(v) for v in cell)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._p = ctypes.c_void_p()
        _l.check(self._lib.demag_setup(ctypes.byref(self._p), *self.n, *self.cell, int(pbc), int(images)))
        self._bind()

    def _bind(self):
        kb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _l.check(self._lib.demag_buffer_bytes(self._p, ctypes.byref(kb), ctypes.byref(wb)))
        Nx, Ny, Nz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _l.check(self._lib.demag_padded_dims(self._p, ctypes.byref(Nx), ctypes.byref(Ny), ctypes.byref(Nz)))
        self.padded = (Nx.value, Ny.value, Nz.value)
        self.kernel_bytes, self.work_bytes = kb.value, wb.value
        with torch.cuda.device(self.device):
            # over-allocate by 256 bytes and align, the library needs 256-byte alignment
            self._kbuf = torch.empty(kb.value + 256, dtype=torch.uint8, device=self.device)
            self._wbuf = torch.empty(wb.value + 256, dtype=torch.uint8, device=self.device)
            _l.check(self._lib.demag_bind(self._p, self._aligned(self._kbuf), self._aligned(self._wbuf), _stream()))

    @staticmethod
    def _aligned(buf):
        a = buf.data_ptr()
        return ctypes.c_void_p((a + 255) & ~255)

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (3, nz, ny, nx)

    @property
    def _vec_shape(self):
        return self.shape

    @property
    def volume(self):
        return self.cell[0] * self.cell[1] * self.cell[2]

    def _check_vec(self, t, name):
        if t.shape != self.shape or t.dtype != torch.float32 or not t.is_contiguous() or t.device != self.device:
            raise ValueError(f"{name}: expected contiguous float32 {self.shape} on {self.device}, "
                             f"got {tuple(t.shape)} {t.dtype} on {t.device}")

    def _ms(self, Ms):
        if isinstance(Ms, torch.Tensor):
            nx, ny, nz = self.n
            if Ms.shape != (nz, ny, nx) or Ms.dtype != torch.float32 or not Ms.is_contiguous():
                raise ValueError("Ms: expected a contiguous float32 (nz, ny, nx) tensor or a float")
            return Ms, 0.0
        return None, float(Ms)

    def field(self, m, Ms, out=None, accumulate=False, energy=False):
        """H_d = -N * (Ms m).  Returns H, or (H, E) with E a 0-d float64 device
        tensor when energy=True."""
        self._check_vec(m, "m")
        if out is None:
            out = torch.empty_like(m)
        else:
            self._check_vec(out, "out")
        msa, mss = self._ms(Ms)
        e = torch.empty((), dtype=torch.float64, device=self.device) if energy else None
        _l.check(self._lib.demag_field(self._p, _ptr(m), _ptr(msa), mss, _ptr(out),
                                       _l.ACCUMULATE if accumulate else 0, _ptr(e), _stream()))
        return (out, e) if energy else out

    def field_2sub(self, mA, mB, MsA, MsB, out=None, accumulate=False, energy=False):
        """Demagnetizing field of the mean magnetization (MsA mA + MsB mB) / 2
        of two sublattices."""
        self._check_vec(mA, "mA")
        self._check_vec(mB, "mB")
        out = torch.empty_like(mA) if out is None else out
        self._check_vec(out, "out")
        e = torch.empty((), dtype=torch.float64, device=self.device) if energy else None
        _l.check(self._lib.demag_field_2sub(self._p, _ptr(mA), _ptr(mB), float(MsA), float(MsB), _ptr(out),
                                            _l.ACCUMULATE if accumulate else 0, _ptr(e), _stream()))
        return (out, e) if energy else out

    def llg_rk4(self, m, Ms, A, alpha, dt, Hext=(0.0, 0.0, 0.0), gamma=0.0, steps=1):
        """`steps` RK4 steps of the LLG equation in place on m (demagnetizing,
        exchange and applied fields); returns m."""
        self._check_vec(m, "m")
        if getattr(self, "_llg_work", None) is None:
            nb = ctypes.c_size_t()
            _l.check(self._lib.demag_llg_workspace_bytes(self._p, ctypes.byref(nb)))
            self._llg_work = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        prm = _l.LlgParams(float(Ms), float(A), float(alpha), float(gamma), float(dt),
                           (ctypes.c_float * 3)(*[float(v) for v in Hext]))
        for _ in range(steps):
            _l.check(self._lib.demag_llg_rk4(self._p, _ptr(m), ctypes.byref(prm), self._aligned(self._llg_work),
                                             _stream()))
        return m

    def energy(self, m, Ms, H):
        """E = -(mu0/2) V sum Ms m . H as a 0-d float64 device tensor."""
        self._check_vec(m, "m")
        self._check_vec(H, "H")
        msa, mss = self._ms(Ms)
        e = torch.empty((), dtype=torch.float64, device=self.device)
        _l.check(self._lib.demag_energy(self._p, _ptr(m), _ptr(msa), mss, _ptr(H), _ptr(e), _stream()))
        return e

    def backward(self, G, Ms, H=None, gE=None, out=None, accumulate=False):
        """grad_m of <G, H_d> + gE * E_demag: Ms * (-N * G - mu0 V gE H)."""
        self._check_vec(G, "G")
        if out is None:
            out = torch.empty_like(G)
        msa, mss = self._ms(Ms)
        if gE is not None:
            gE = gE.to(device=self.device, dtype=torch.float64).reshape(()).contiguous()
            self._check_vec(H, "H")
        _l.check(self._lib.demag_backward(self._p, _ptr(G), _ptr(msa), mss, _ptr(H) if gE is not None else None,
                                          _ptr(gE), _ptr(out), _l.ACCUMULATE if accumulate else 0, _stream()))
        return out

    def __del__(self):
        p = getattr(self, "_p", None)
        if p is not None and p.value:
            self._lib.demag_destroy(p)
            self._p = None


class DemagBatch(_Schedules):
    """Batch of meshes: meshes = [((nx, ny, nz), (dx, dy, dz)), ...], with
    optional origins (lower corners, metres) and group ids (meshes sharing an
    id >= 0 are coupled layers, Sec. 3 Eq. 4; others independent).
    Vectors of all meshes are concatenated (mesh order, each SoA
    [3][nz][ny][nx]) into one flat float32 tensor of `total` elements;
    `view(x, i)` returns mesh i's block.  Meshes of equal geometry share one
    kernel spectrum and run through the same launches."""

    def __init__(self, meshes, device=None, origins=None, groups=None, pbc=0, images=0):
        self._lib = _l.load()
        self.meshes = [(tuple(int(v) for v in n), tuple(float(v) for v in h)) for n, h in meshes]
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        k = len(self.meshes)
        dims = (ctypes.c_int * (3 * k))(*[v for n, _ in self.meshes for v in n])
        cells = (ctypes.c_double * (3 * k))(*[v for _, h in self.meshes for v in h])
        orig = (ctypes.c_double * (3 * k))(*[float(v) for o in origins for v in o]) if origins is not None else None
        grp = (ctypes.c_int * k)(*[int(v) for v in groups]) if groups is not None else None
        self._p = ctypes.c_void_p()
        _l.check(self._lib.demag_setup_batch(ctypes.byref(self._p), k, dims, cells, orig, grp, int(pbc), int(images)))
        nm, tot = ctypes.c_int(), ctypes.c_size_t()
        offs = (ctypes.c_longlong * k)()
        _l.check(self._lib.demag_batch_layout(self._p, ctypes.byref(nm), offs, ctypes.byref(tot)))
        self.offsets = [int(o) for o in offs]
        self.total = tot.value
        kb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _l.check(self._lib.demag_buffer_bytes(self._p, ctypes.byref(kb), ctypes.byref(wb)))
        with torch.cuda.device(self.device):
            self._kbuf = torch.empty(kb.value + 256, dtype=torch.uint8, device=self.device)
            self._wbuf = torch.empty(wb.value + 256, dtype=torch.uint8, device=self.device)
            _l.check(self._lib.demag_bind(self._p, DemagPlan._aligned(self._kbuf), DemagPlan._aligned(self._wbuf),
                                          _stream()))

    @property
    def _vec_shape(self):
        return (self.total,)

    def view(self, x, i):
        (nx, ny, nz), _ = self.meshes[i]
        o = self.offsets[i]
        return x[o:o + 3 * nx * ny * nz].view(3, nz, ny, nx)

    def _check(self, t, name):
        if t.shape != (self.total,) or t.dtype != torch.float32 or not t.is_contiguous() or t.device != self.device:
            raise ValueError(f"{name}: expected a contiguous float32 ({self.total},) tensor on {self.device}")

    def field(self, m, Ms, out=None, accumulate=False, energy=False):
        """Fields of all meshes; Ms is a float or a float32 tensor of one value per mesh."""
        self._check(m, "m")
        out = torch.empty_like(m) if out is None else out
        self._check(out, "out")
        msa, mss = (Ms, 0.0) if isinstance(Ms, torch.Tensor) else (None, float(Ms))
        e = torch.empty(len(self.meshes), dtype=torch.float64, device=self.device) if energy else None
        _l.check(self._lib.demag_field_batch(self._p, _ptr(m), _ptr(msa), mss, _ptr(out),
                                             _l.ACCUMULATE if accumulate else 0, _ptr(e), _stream()))
        return (out, e) if energy else out

    def backward(self, G, Ms, H=None, gE=None, out=None):
        self._check(G, "G")
        out = torch.empty_like(G) if out is None else out
        msa, mss = (Ms, 0.0) if isinstance(Ms, torch.Tensor) else (None, float(Ms))
        _l.check(self._lib.demag_backward_batch(self._p, _ptr(G), _ptr(msa), mss, _ptr(H) if gE is not None else None,
                                                _ptr(gE), _ptr(out), 0, _stream()))
        return out

    def __del__(self):
        p = getattr(self, "_p", None)
        if p is not None and p.value:
            self._lib.demag_destroy(p)
            self._p = None


class OerstedPlan(DemagPlan):
    """Oersted field of a current density on one mesh of n = (nx, ny, nz)
    cells of size cell (metres): H = K * J with the cell-averaged Biot-Savart
    kernel (include/demag.h, demag_setup_oersted).  pbc / images as for
    DemagPlan.  Builds the kernel spectrum on construction; schedules and the
    tuner as for DemagPlan."""

    def __init__(self, n, cell, device=None, pbc=0, images=0):
        self._lib = _l.load()
        self.n = tuple(int(v) for v in n)
        self.cell = tuple(float(v) for v in cell)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._p = ctypes.c_void_p()
        _l.check(self._lib.demag_setup_oersted(ctypes.byref(self._p), *self.n, *self.cell, int(pbc), int(images)))
        self._bind()

    def field(self, J, scale=1.0, out=None, accumulate=False):
        """H (A/m) of the current density J (A/m^2, SoA (3, nz, ny, nx)),
        times scale."""
        self._check_vec(J, "J")
        if out is None:
            out = torch.empty_like(J)
        else:
            self._check_vec(out, "out")
        _l.check(self._lib.demag_oersted_field(self._p, _ptr(J), float(scale), _ptr(out),
                                               _l.ACCUMULATE if accumulate else 0, _stream()))
        return out

    def field_2sub(self, *a, **k):
        raise TypeError("an Oersted plan computes oersted fields only")

    llg_rk4 = energy = backward = field_2sub


class OerstedFunction(torch.autograd.Function):
    """H = K * J with its backward: J -> H is self-adjoint, so the gradient
    of <G, H> with respect to J is K * G, the same call."""

    @staticmethod
    def forward(ctx, J, plan, scale):
        ctx.plan, ctx.scale = plan, scale
        return plan.field(J.contiguous(), scale)

    @staticmethod
    def backward(ctx, gH):
        return ctx.plan.field(gH.contiguous(), ctx.scale), None, None


def oersted(J, plan, scale=1.0):
    """Differentiable Oersted field of the current density J."""
    return OerstedFunction.apply(J, plan, scale)


class DemagFunction(torch.autograd.Function):
    """(H_d, E) = demag(m) for M = Ms m with a hand-written backward: the
    operator is self-adjoint, so the gradient of <G, H_d> is the same
    convolution applied to G, and that of E is -mu0 V Ms H_d."""

    @staticmethod
    def forward(ctx, m, plan, Ms):
        H, E = plan.field(m.contiguous(), Ms, energy=True)
        ctx.plan, ctx.Ms = plan, Ms
        ctx.save_for_backward(H)
        return H, E

    @staticmethod
    def backward(ctx, gH, gE):
        (H,) = ctx.saved_tensors
        if gH is None:
            gH = torch.zeros_like(H)
        grad_m = ctx.plan.backward(gH.contiguous(), ctx.Ms, H=H, gE=gE)
        return grad_m, None, None


def demag(m, plan, Ms):
    """Differentiable (H_d, E_demag) of a unit magnetization m."""
    return DemagFunction.apply(m, plan, Ms)
