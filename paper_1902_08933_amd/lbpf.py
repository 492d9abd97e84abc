"""ctypes binding of liblbpf.so (see include/lbpf.h): argument marshalling only.

Every step of the solver runs in the HIP library. PyTorch supplies device memory (the
workspace and field tensors) and the current HIP stream. There is no CPU fallback: if the
library is missing or no GPU is visible, construction raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbpf.so")

FIELDS = {"phi": 0, "rho": 1, "ux": 2, "uy": 3, "p": 4, "mu": 5}
VARIANTS = {"qim": 0, "im": 1}
PSCHEMES = {"eq28": 0, "eq28_paper_g0": 1, "eq29": 2}
FSURF = {"mu_grad_phi": 0, "neg_phi_grad_mu": 1}
VISC = {"inverse_linear": 0, "step": 1}
BCS = {"periodic": 0, "walls_y": 1}
STATUS = {0: "LBPF_OK", -1: "LBPF_E_INVALID", -2: "LBPF_E_HIP", -3: "LBPF_E_NOMEM",
          -4: "LBPF_E_UNSTABLE", -5: "LBPF_E_STATE"}


class LbpfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("pscheme", ctypes.c_int32), ("fsurf", ctypes.c_int32), ("visc", ctypes.c_int32),
                ("bc", ctypes.c_int32), ("clamp_props", ctypes.c_int32),
                ("rho_A", ctypes.c_double), ("rho_B", ctypes.c_double),
                ("nu_A", ctypes.c_double), ("nu_B", ctypes.c_double),
                ("sigma", ctypes.c_double), ("W", ctypes.c_double), ("M_phi", ctypes.c_double),
                ("tau_h", ctypes.c_double), ("force_x", ctypes.c_double),
                ("force_y", ctypes.c_double), ("gravity", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("sum_phi", ctypes.c_double), ("sum_rho", ctypes.c_double),
                ("max_u", ctypes.c_double), ("nonfinite", ctypes.c_int64),
                ("step", ctypes.c_int64)]


# every symbol include/lbpf.h declares, with (restype, argtypes)
_V = ctypes.c_void_p
_S = ctypes.c_int
SIGNATURES = {
    "lbpf_workspace_size": (_S, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
    "lbpf_create": (_S, [ctypes.POINTER(Params), _V, ctypes.c_size_t, _V, ctypes.POINTER(_V)]),
    "lbpf_init": (_S, [_V, _V, _V, _V, _V]),
    "lbpf_step": (_S, [_V, ctypes.c_int64]),
    "lbpf_read": (_S, [_V, ctypes.c_int32, _V]),
    "lbpf_diagnostics": (_S, [_V, ctypes.POINTER(Diag)]),
    "lbpf_laplace_dp": (_S, [_V, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                             ctypes.POINTER(ctypes.c_double)]),
    "lbpf_field_stats": (_S, [_V, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "lbpf_field_stats_many": (_S, [_V, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "lbpf_diagnostics_noalloc": (_S, [_V, ctypes.POINTER(Diag)]),
    "lbpf_state_size": (_S, [_V, ctypes.POINTER(ctypes.c_size_t)]),
    "lbpf_save_state": (_S, [_V, _V]),
    "lbpf_load_state": (_S, [_V, _V]),
    "lbpf_set_stream": (_S, [_V, _V]),
    "lbpf_set_tile": (_S, [_V, ctypes.c_int32]),
    "lbpf_autotune": (_S, [_V, ctypes.c_int32, _V, ctypes.POINTER(ctypes.c_float),
                           ctypes.POINTER(ctypes.c_int32)]),
    "lbpf_get_tile": (ctypes.c_int32, [_V]),
    "lbpf_tile_count": (ctypes.c_int32, []),
    "lbpf_tile_shape": (_S, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "lbpf_step_count": (ctypes.c_int64, [_V]),
    "lbpf_bw_probe": (_S, [ctypes.c_int32, _V, _V, ctypes.c_size_t, ctypes.c_int32, _V]),
    "lbpf_destroy": (_S, [_V]),
    "lbpf_batch_workspace_size": (_S, [ctypes.c_int32, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
    "lbpf_batch_create": (_S, [ctypes.c_int32, ctypes.POINTER(Params), _V, ctypes.c_size_t, _V,
                               ctypes.POINTER(_V)]),
    "lbpf_batch_init": (_S, [_V, ctypes.c_int32, _V, _V, _V, _V]),
    "lbpf_batch_step": (_S, [_V, ctypes.c_int64]),
    "lbpf_batch_step_each": (_S, [_V, ctypes.c_int64]),
    "lbpf_batch_status": (_S, [_V, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Diag)]),
    "lbpf_batch_instance": (_V, [_V, ctypes.c_int32]),
    "lbpf_batch_count": (ctypes.c_int32, [_V]),
    "lbpf_batch_set_tile": (_S, [_V, ctypes.c_int32]),
    "lbpf_batch_get_tile": (ctypes.c_int32, [_V]),
    "lbpf_batch_state_size": (_S, [_V, ctypes.POINTER(ctypes.c_size_t)]),
    "lbpf_batch_autotune": (_S, [_V, ctypes.c_int32, _V, ctypes.POINTER(ctypes.c_float),
                                 ctypes.POINTER(ctypes.c_int32)]),
    "lbpf_batch_step_count": (ctypes.c_int64, [_V]),
    "lbpf_batch_destroy": (_S, [_V]),
    "lbpf_batch_last_error": (ctypes.c_char_p, [_V]),
    "lbpf_status_string": (ctypes.c_char_p, [_S]),
    "lbpf_last_error": (ctypes.c_char_p, [_V]),
    "lbpf_create_error": (ctypes.c_char_p, []),
}

_lib = None


def library(path=LIB_PATH):
    """Load liblbpf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1902_08933_amd.build`"
                           " (or __graft_entry__.build())")
    # PyTorch ships its own HIP runtime and asks for it by an unversioned name. Loaded first,
    # that runtime also satisfies this library's libamdhip64.so.7; loaded after this library,
    # it would be a second HIP (and HSA) runtime in the process, and this library's launches
    # then find no device. So torch is imported before the library is opened.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def make_params(cfg):
    """Params from a workload dict (keys as in paper_1902_08933_amd.workloads)."""
    p = Params()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.variant = VARIANTS[cfg.get("variant", "qim")]
    p.pscheme = PSCHEMES[cfg.get("pscheme", "eq28")]
    p.fsurf = FSURF[cfg.get("fsurf", "mu_grad_phi")]
    p.visc = VISC[cfg.get("visc", "inverse_linear")]
    p.bc = BCS[cfg.get("bc", "periodic")]
    p.clamp_props = int(bool(cfg.get("clamp_props", False)))
    for k in ("rho_A", "rho_B", "nu_A", "nu_B", "sigma", "W", "M_phi", "tau_h"):
        setattr(p, k, float(cfg[k]))
    p.force_x = float(cfg.get("force_x", 0.0))
    p.force_y = float(cfg.get("force_y", 0.0))
    p.gravity = float(cfg.get("gravity", 0.0))
    return p


def _check(status, handle=None):
    if status != 0:
        lib = library()
        msg = lib.lbpf_last_error(handle) if handle else lib.lbpf_create_error()
        raise LbpfError(status, (msg or b"").decode())


def workspace_size(cfg):
    lib = library()
    n = ctypes.c_size_t()
    _check(lib.lbpf_workspace_size(ctypes.byref(make_params(cfg)), ctypes.byref(n)))
    return n.value


def tile_shapes():
    lib = library()
    out = []
    for i in range(lib.lbpf_tile_count()):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.lbpf_tile_shape(i, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        out.append((a.value, b.value, c.value))
    return out


def bw_probe(mode, src, dst, nbytes, blocks=0, stream=None):
    """Launch the bandwidth probe (mode 0 copy, 1 read, 2 write) on torch tensors."""
    import torch
    lib = library()
    st = (stream or torch.cuda.current_stream()).cuda_stream
    _check(lib.lbpf_bw_probe(int(mode), ctypes.c_void_p(src.data_ptr()) if src is not None else None,
                             ctypes.c_void_p(dst.data_ptr()), ctypes.c_size_t(nbytes), int(blocks),
                             ctypes.c_void_p(st)))


def _dev_ptr(t, torch, shape=None):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("fields must be contiguous float32 tensors on the GPU")
    if shape is not None and tuple(t.shape) != shape:
        raise ValueError(f"field shape {tuple(t.shape)} != {shape}")
    return ctypes.c_void_p(t.data_ptr())


class Simulation:
    """One simulation on one GPU: init fields, step N, read phi/rho/u/p/mu."""

    def __init__(self, cfg, device="cuda"):
        import torch
        self.torch = torch
        self.lib = library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lbpf solver runs only on the GPU")
        self.device = torch.device(device)
        self.cfg = dict(cfg)
        self.params = make_params(cfg)
        self.nx, self.ny = self.params.nx, self.params.ny
        nbytes = workspace_size(cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        h = ctypes.c_void_p()
        _check(self.lib.lbpf_create(ctypes.byref(self.params),
                                    ctypes.c_void_p(self.workspace.data_ptr()),
                                    ctypes.c_size_t(nbytes), ctypes.c_void_p(stream),
                                    ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.lbpf_destroy(h)
            self._h = None

    def _c(self, status):
        _check(status, self._h)

    def _as_field(self, a):
        torch = self.torch
        if a is None:
            return None
        t = torch.as_tensor(a, dtype=torch.float32, device=self.device).contiguous()
        if tuple(t.shape) != (self.ny, self.nx):
            raise ValueError(f"field shape {tuple(t.shape)} != {(self.ny, self.nx)}")
        return t

    def init(self, phi, ux=None, uy=None, p=None):
        fields = [self._as_field(a) for a in (phi, ux, uy, p)]
        ptrs = [_dev_ptr(t, self.torch) for t in fields]
        self._c(self.lib.lbpf_init(self._h, *ptrs))
        self.torch.cuda.current_stream(self.device).synchronize()
        return self

    def step(self, n=1):
        self._c(self.lib.lbpf_step(self._h, int(n)))
        return self

    def read(self, field, out=None):
        t = out if out is not None else self.torch.empty((self.ny, self.nx), dtype=self.torch.float32,
                                                         device=self.device)
        self._c(self.lib.lbpf_read(self._h, FIELDS[field], _dev_ptr(t, self.torch, (self.ny, self.nx))))
        return t

    def field_stats(self, field):
        """FP64 mean, standard deviation and largest magnitude of a field (lbpf_field_stats)"""
        out = (ctypes.c_double * 3)()
        self._c(self.lib.lbpf_field_stats(self._h, FIELDS[field], out))
        return {"mean": out[0], "std": out[1], "max_abs": out[2]}

    def field_stats_many(self, fields):
        """field_stats of several fields with one synchronization (lbpf_field_stats_many):
        {name: {mean, std, max_abs}}"""
        names = list(fields)
        ids = (ctypes.c_int32 * len(names))(*[FIELDS[f] for f in names])
        out = (ctypes.c_double * (3 * len(names)))()
        self._c(self.lib.lbpf_field_stats_many(self._h, len(names), ids, out))
        return {f: {"mean": out[3 * k], "std": out[3 * k + 1], "max_abs": out[3 * k + 2]} for k, f in enumerate(names)}

    def diagnostics(self, check=True):
        d = Diag()
        st = self.lib.lbpf_diagnostics(self._h, ctypes.byref(d))
        if check:
            self._c(st)
        return dict(sum_phi=d.sum_phi, sum_rho=d.sum_rho, max_u=d.max_u,
                    nonfinite=d.nonfinite, step=d.step, status=st)

    def laplace_dp(self, xc, yc, R):
        v = ctypes.c_double()
        self._c(self.lib.lbpf_laplace_dp(self._h, float(xc), float(yc), float(R), ctypes.byref(v)))
        return v.value

    def state_size(self):
        n = ctypes.c_size_t()
        self._c(self.lib.lbpf_state_size(self._h, ctypes.byref(n)))
        return n.value

    def save_state(self, out=None):
        buf = out if out is not None else self.torch.empty(self.state_size(), dtype=self.torch.uint8,
                                                           device=self.device)
        self._c(self.lib.lbpf_save_state(self._h, ctypes.c_void_p(buf.data_ptr())))
        return buf

    def load_state(self, buf):
        if buf.numel() < self.state_size() or not buf.is_cuda:
            raise ValueError("checkpoint buffer too small or not on the GPU")
        self._c(self.lib.lbpf_load_state(self._h, ctypes.c_void_p(buf.data_ptr())))
        return self

    def set_tile(self, index):
        self._c(self.lib.lbpf_set_tile(self._h, int(index)))
        return self

    def autotune(self, trial_steps=20):
        """Time every strip shape on this grid, keep the fastest; the state is restored."""
        n = self.lib.lbpf_tile_count()
        ms = (ctypes.c_float * n)()
        best = ctypes.c_int32()
        scratch = self.torch.empty(self.state_size(), dtype=self.torch.uint8, device=self.device)
        self._c(self.lib.lbpf_autotune(self._h, int(trial_steps), ctypes.c_void_p(scratch.data_ptr()),
                                       ms, ctypes.byref(best)))
        return best.value, list(ms)

    def set_stream(self, stream):
        self._c(self.lib.lbpf_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))
        return self

    @property
    def tile(self):
        return int(self.lib.lbpf_get_tile(self._h))

    @property
    def step_count(self):
        return int(self.lib.lbpf_step_count(self._h))


class _InstanceView(Simulation):
    """A batch instance seen through the single-simulation calls (read, diagnostics, ...)."""

    def __init__(self, batch, idx):  # noqa: D107 - no workspace of its own
        self.torch = batch.torch
        self.lib = batch.lib
        self.device = batch.device
        self.cfg = batch.cfgs[idx]
        self.params = make_params(self.cfg)
        self.nx, self.ny = self.params.nx, self.params.ny
        self._h = ctypes.c_void_p(self.lib.lbpf_batch_instance(batch._h, idx))
        self._batch = batch  # keeps the owner alive

    def __del__(self):
        pass  # the batch owns the handle

    def init(self, *a, **k):
        raise RuntimeError("initialize batch instances with Batch.init")

    def step(self, n=1):
        raise RuntimeError("step batch instances with Batch.step")


class Batch:
    """Many independent simulations advanced by one persistent launch per step."""

    def __init__(self, cfgs, device="cuda"):
        import torch
        self.torch = torch
        self.lib = library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lbpf solver runs only on the GPU")
        self.device = torch.device(device)
        self.cfgs = [dict(c) for c in cfgs]
        n = len(self.cfgs)
        self._params = (Params * n)(*[make_params(c) for c in self.cfgs])
        nb = ctypes.c_size_t()
        _check(self.lib.lbpf_batch_workspace_size(n, self._params, ctypes.byref(nb)))
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        h = ctypes.c_void_p()
        _check(self.lib.lbpf_batch_create(n, self._params, ctypes.c_void_p(self.workspace.data_ptr()),
                                          ctypes.c_size_t(nb.value), ctypes.c_void_p(stream),
                                          ctypes.byref(h)))
        self._h = h
        self.n = n

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.lbpf_batch_destroy(h)
            self._h = None

    def _c(self, status):
        if status != 0:
            raise LbpfError(status, (self.lib.lbpf_batch_last_error(self._h) or b"").decode())

    def init(self, idx, phi, ux=None, uy=None, p=None):
        c = self.cfgs[idx]
        shape = (int(c["ny"]), int(c["nx"]))
        ts = []
        for a in (phi, ux, uy, p):
            if a is None:
                ts.append(None)
                continue
            t = self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device).contiguous()
            if tuple(t.shape) != shape:
                raise ValueError(f"instance {idx}: field shape {tuple(t.shape)} != {shape}")
            ts.append(t)
        ptrs = [None if t is None else ctypes.c_void_p(t.data_ptr()) for t in ts]
        self._c(self.lib.lbpf_batch_init(self._h, int(idx), *ptrs))
        self.torch.cuda.current_stream(self.device).synchronize()
        return self

    def step(self, n=1):
        self._c(self.lib.lbpf_batch_step(self._h, int(n)))
        return self

    def step_each(self, n=1):
        self._c(self.lib.lbpf_batch_step_each(self._h, int(n)))
        return self

    def status(self):
        flags = (ctypes.c_int32 * self.n)()
        diags = (Diag * self.n)()
        self._c(self.lib.lbpf_batch_status(self._h, flags, diags))
        return list(flags), [dict(sum_phi=d.sum_phi, sum_rho=d.sum_rho, max_u=d.max_u,
                                  nonfinite=d.nonfinite, step=d.step) for d in diags]

    def instance(self, idx):
        return _InstanceView(self, idx)

    def set_tile(self, index):
        self._c(self.lib.lbpf_batch_set_tile(self._h, int(index)))
        return self

    @property
    def tile(self):
        return int(self.lib.lbpf_batch_get_tile(self._h))

    @property
    def step_count(self):
        return int(self.lib.lbpf_batch_step_count(self._h))

    def autotune(self, trial_steps=10):
        nb = ctypes.c_size_t()
        self._c(self.lib.lbpf_batch_state_size(self._h, ctypes.byref(nb)))
        scratch = self.torch.empty(nb.value, dtype=self.torch.uint8, device=self.device)
        n = self.lib.lbpf_tile_count()
        ms = (ctypes.c_float * n)()
        best = ctypes.c_int32()
        self._c(self.lib.lbpf_batch_autotune(self._h, int(trial_steps), ctypes.c_void_p(scratch.data_ptr()),
                                             ms, ctypes.byref(best)))
        return best.value, list(ms)


class UNetCfg(ctypes.Structure):
    _fields_ = [("in_ch", ctypes.c_int32), ("base_ch", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_h", ctypes.c_int32),
                ("max_w", ctypes.c_int32), ("train", ctypes.c_int32),
                ("wgrad_chunks", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


_PF = ctypes.POINTER(ctypes.c_float)
_PD = ctypes.POINTER(ctypes.c_double)
SIGNATURES.update({
    "lbpf_unet_workspace_size": (_S, [ctypes.POINTER(UNetCfg), ctypes.POINTER(ctypes.c_size_t)]),
    "lbpf_unet_create": (_S, [ctypes.POINTER(UNetCfg), _V, ctypes.c_size_t, _V, ctypes.POINTER(_V)]),
    "lbpf_unet_param_count": (ctypes.c_int64, [_V]),
    "lbpf_unet_layer": (_S, [_V, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                             ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "lbpf_unet_get_params": (_S, [_V, _V]),
    "lbpf_unet_set_params": (_S, [_V, _V]),
    "lbpf_unet_set_loss_weights": (_S, [_V, _PF]),
    "lbpf_unet_forward": (_S, [_V, _V, _V, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "lbpf_unet_loss_grad": (_S, [_V, _V, _V, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _PD, _V]),
    "lbpf_unet_train_step": (_S, [_V, _V, _V, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_float, _PD]),
    "lbpf_unet_destroy": (_S, [_V]),
    "lbpf_unet_last_error": (ctypes.c_char_p, [_V]),
    "lbpf_mfma_probe": (_S, [ctypes.c_int32, _V, _V, _V, _V]),
    "lbpf_unet_conv_probe": (_S, [_V, ctypes.POINTER(ctypes.c_int32), _V]),
    "lbpf_unet_wgrad_probe": (_S, [ctypes.c_int32, _V, _V, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _V, _V, _V, _V, _V]),
    "lbpf_fields_to_nhwc": (_S, [_V, _V, _PF, _PF]),
    "lbpf_init_from_nhwc": (_S, [_V, _V, _PF, _PF, ctypes.c_int64]),
})


def _f4(v):
    return (ctypes.c_float * 4)(*[float(a) for a in v])


def fields_to_nhwc(sim, shift, scale, out=None):
    """Current fields (phi, u_x, u_y, p) of a simulation as normalized NHWC [ny, nx, 4]."""
    torch = sim.torch
    t = out if out is not None else torch.empty((sim.ny, sim.nx, 4), dtype=torch.float32, device=sim.device)
    sim._c(sim.lib.lbpf_fields_to_nhwc(sim._h, ctypes.c_void_p(t.data_ptr()), _f4(shift), _f4(scale)))
    return t


def init_from_nhwc(sim, src, shift, scale, step=None):
    """Replace the state of a simulation by equilibria of normalized NHWC fields at time level
    `step` (default: the current step count)."""
    st = sim.step_count if step is None else int(step)
    sim._c(sim.lib.lbpf_init_from_nhwc(sim._h, ctypes.c_void_p(src.data_ptr()), _f4(shift), _f4(scale), st))
    return sim


def mfma_probe(A_bf16_bits, B_bf16_bits, D, k=16):
    """One 16x16xk MFMA product (k = 16 or 32); A, B int16 tensors holding BF16 bits."""
    import torch
    lib = library()
    st = lib.lbpf_mfma_probe(int(k), ctypes.c_void_p(A_bf16_bits.data_ptr()), ctypes.c_void_p(B_bf16_bits.data_ptr()),
                             ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != 0:
        raise LbpfError(st, "mfma probe")
    return D


class ConvDesc(ctypes.Structure):
    """lbpf_unet_conv_desc"""
    _fields_ = [(k, ctypes.c_int32) for k in ("ks", "relu", "n", "h", "w", "cin", "cl", "cout", "xin_c", "rc")] + \
               [(k, ctypes.c_void_p) for k in ("x", "xl", "xin", "wt", "bias", "y", "yp", "yf", "res", "pred",
                                               "hw", "hb")]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def conv_probe(ks, relu, n, h, w, cin, cout, wt, x=None, xl=None, cl=0, xin=None, bias=None, y=None, yp=None,
               yf=None, res=None, pred=None, hw=None, hb=None):
    """One convolution by the network's kernels (lbpf_unet_conv_probe); tensors are contiguous
    NHWC device arrays (bf16 ones as int16 bits). Returns the kernel variant (first, cot, pfw)."""
    import torch
    d = ConvDesc()
    d.ks, d.relu, d.n, d.h, d.w, d.cin, d.cl, d.cout = ks, int(bool(relu)), n, h, w, cin, cl, cout
    d.xin_c = xin.shape[-1] if xin is not None else 0
    d.rc = res.shape[-1] if res is not None else 0
    for k, t in (("x", x), ("xl", xl), ("xin", xin), ("wt", wt), ("bias", bias), ("y", y), ("yp", yp),
                 ("yf", yf), ("res", res), ("pred", pred), ("hw", hw), ("hb", hb)):
        setattr(d, k, t.data_ptr() if t is not None else None)
    var = (ctypes.c_int32 * 3)()
    st = library().lbpf_unet_conv_probe(ctypes.byref(d), var, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != 0:
        raise LbpfError(st, "conv probe")
    return tuple(var)


def wgrad_probe(ks, dy, x, n, h, w, cin, cout, max_chunks=64):
    """Weight and bias gradients of one convolution by the network's kernels; returns (dw, db)
    as FP32 device tensors [cout, ks*ks, cin] and [cout]."""
    import torch
    dev = dy.device
    part = torch.empty(max_chunks * cout * ks * ks * cin, dtype=torch.float32, device=dev)
    bpart = torch.empty(max_chunks * cout, dtype=torch.float32, device=dev)
    dw = torch.empty((cout, ks * ks, cin), dtype=torch.float32, device=dev)
    db = torch.empty(cout, dtype=torch.float32, device=dev)
    st = library().lbpf_unet_wgrad_probe(ks, _ptr(dy), _ptr(x), n, h, w, cin, cout, max_chunks, _ptr(part),
                                         _ptr(bpart), _ptr(dw), _ptr(db),
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != 0:
        raise LbpfError(st, "wgrad probe")
    return dw, db


class UNet:
    """The learned surrogate (see include/lbpf.h): forward, loss/gradient, Adam step."""

    def __init__(self, in_ch=4, base_ch=32, max_batch=1, max_h=256, max_w=256, train=True,
                 wgrad_chunks=0, seed=0, device="cuda"):
        import torch
        self.torch = torch
        self.lib = library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the surrogate runs only on the GPU")
        self.device = torch.device(device)
        self.cfg = UNetCfg(in_ch, base_ch, max_batch, max_h, max_w, int(bool(train)), wgrad_chunks, 0, seed)
        nb = ctypes.c_size_t()
        st = self.lib.lbpf_unet_workspace_size(ctypes.byref(self.cfg), ctypes.byref(nb))
        if st != 0:
            raise LbpfError(st, self.lib.lbpf_unet_last_error(None).decode())
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        st = self.lib.lbpf_unet_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.workspace.data_ptr()),
                                       nb, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream),
                                       ctypes.byref(h))
        if st != 0:
            raise LbpfError(st, self.lib.lbpf_unet_last_error(None).decode())
        self._h = h
        self.in_ch = in_ch
        self.nparam = int(self.lib.lbpf_unet_param_count(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.lbpf_unet_destroy(h)
            self._h = None

    def _c(self, st):
        if st != 0:
            raise LbpfError(st, (self.lib.lbpf_unet_last_error(self._h) or b"").decode())

    def layers(self):
        out = []
        for i in range(8):
            wo, bo = ctypes.c_int64(), ctypes.c_int64()
            co, ks, ci = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            self._c(self.lib.lbpf_unet_layer(self._h, i, ctypes.byref(wo), ctypes.byref(bo), ctypes.byref(co),
                                             ctypes.byref(ks), ctypes.byref(ci)))
            out.append(dict(woff=wo.value, boff=bo.value, cout=co.value, ks=ks.value, cin=ci.value))
        return out

    def get_params(self):
        t = self.torch.empty(self.nparam, dtype=self.torch.float32, device=self.device)
        self._c(self.lib.lbpf_unet_get_params(self._h, ctypes.c_void_p(t.data_ptr())))
        return t

    def set_params(self, t):
        t = t.to(self.device, self.torch.float32).contiguous()
        self._c(self.lib.lbpf_unet_set_params(self._h, ctypes.c_void_p(t.data_ptr())))

    def set_loss_weights(self, w):
        arr = (ctypes.c_float * 16)(*([float(v) for v in w] + [0.0] * (16 - len(w))))
        self._c(self.lib.lbpf_unet_set_loss_weights(self._h, arr))

    def _chk(self, x):
        if not (x.is_cuda and x.dtype == self.torch.float32 and x.is_contiguous() and x.dim() == 4
                and x.shape[3] == self.in_ch):
            raise ValueError("expected a contiguous float32 NHWC tensor on the GPU")
        return x.shape[0], x.shape[1], x.shape[2]

    def forward(self, x, out=None):
        n, h, w = self._chk(x)
        y = out if out is not None else self.torch.empty_like(x)
        self._c(self.lib.lbpf_unet_forward(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                           n, h, w))
        return y

    def loss_grad(self, x, target):
        n, h, w = self._chk(x)
        self._chk(target)
        g = self.torch.empty(self.nparam, dtype=self.torch.float32, device=self.device)
        loss = ctypes.c_double()
        self._c(self.lib.lbpf_unet_loss_grad(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                             n, h, w, ctypes.byref(loss), ctypes.c_void_p(g.data_ptr())))
        return loss.value, g

    def train_step(self, x, target, lr):
        n, h, w = self._chk(x)
        self._chk(target)
        loss = ctypes.c_double()
        self._c(self.lib.lbpf_unet_train_step(self._h, ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(target.data_ptr()), n, h, w, float(lr),
                                              ctypes.byref(loss)))
        return loss.value


# ---- generalized single-phase model with a mass source (lbpf_sp_* of include/lbpf.h) --------

class SpParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("model", ctypes.c_int32),
                ("pscheme", ctypes.c_int32), ("full", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("nu", ctypes.c_double), ("xi", ctypes.c_double), ("rho0", ctypes.c_double),
                ("drag", ctypes.c_double), ("scheme", ctypes.c_int32), ("pad", ctypes.c_int32)]


SP_MODELS = {"nearly_incompressible": 0, "incompressible": 1}
SP_FIELDS = {"rho": 0, "ux": 1, "uy": 2, "p": 3}
SIGNATURES.update({
    "lbpf_sp_workspace_size": (_S, [ctypes.POINTER(SpParams), ctypes.POINTER(ctypes.c_size_t)]),
    "lbpf_sp_create": (_S, [ctypes.POINTER(SpParams), _V, ctypes.c_size_t, _V, ctypes.POINTER(_V)]),
    "lbpf_sp_init": (_S, [_V, _V, _V, _V, _V, _V, _V]),
    "lbpf_sp_step": (_S, [_V, ctypes.c_int64]),
    "lbpf_sp_read": (_S, [_V, ctypes.c_int32, _V]),
    "lbpf_sp_sums": (_S, [_V, _PD]),
    "lbpf_sp_step_count": (ctypes.c_int64, [_V]),
    "lbpf_sp_destroy": (_S, [_V]),
    "lbpf_sp_last_error": (ctypes.c_char_p, [_V]),
})


def make_sp_params(cfg):
    """SpParams from a workload dict (keys as in workloads.single_phase_source)."""
    p = SpParams()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.model = SP_MODELS[cfg["model"]]
    p.pscheme = {"eq28": 0, "eq29": 1}[cfg.get("pscheme", "eq28")]
    p.full = int(bool(cfg.get("full", True)))
    p.bc = BCS[cfg.get("bc", "periodic")]
    p.nu = float(cfg["nu"])
    p.xi = float(cfg.get("xi", 0.0))
    p.rho0 = float(cfg.get("rho0", 1.0))
    p.drag = float(cfg.get("drag", 0.0))
    p.scheme = {"eq24": 0, "remark4": 1}[cfg.get("scheme", "eq24")]
    return p


class SinglePhase:
    """One simulation of the generalized single-phase model on one GPU: init (density or
    pressure, velocity, source and force fields), step N, read rho/u/p, FP64 sums."""

    def __init__(self, cfg, device="cuda"):
        import torch
        self.torch = torch
        self.lib = library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lbpf solver runs only on the GPU")
        self.device = torch.device(device)
        self.cfg = dict(cfg)
        self.params = make_sp_params(cfg)
        self.nx, self.ny = self.params.nx, self.params.ny
        nb = ctypes.c_size_t()
        st = self.lib.lbpf_sp_workspace_size(ctypes.byref(self.params), ctypes.byref(nb))
        if st != 0:
            raise LbpfError(st, (self.lib.lbpf_sp_last_error(None) or b"").decode())
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        h = ctypes.c_void_p()
        st = self.lib.lbpf_sp_create(ctypes.byref(self.params), ctypes.c_void_p(self.workspace.data_ptr()),
                                     ctypes.c_size_t(nb.value), ctypes.c_void_p(stream), ctypes.byref(h))
        if st != 0:
            raise LbpfError(st, (self.lib.lbpf_sp_last_error(None) or b"").decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.lbpf_sp_destroy(h)
            self._h = None

    def _c(self, st):
        if st != 0:
            raise LbpfError(st, (self.lib.lbpf_sp_last_error(self._h) or b"").decode())

    def _as_field(self, a):
        if a is None:
            return None
        t = self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device).contiguous()
        if tuple(t.shape) != (self.ny, self.nx):
            raise ValueError(f"field shape {tuple(t.shape)} != {(self.ny, self.nx)}")
        return t

    def init(self, a0=None, ux=None, uy=None, S=None, Fx=None, Fy=None):
        ts = [self._as_field(a) for a in (a0, ux, uy, S, Fx, Fy)]
        self._c(self.lib.lbpf_sp_init(self._h, *[ctypes.c_void_p(t.data_ptr()) if t is not None else None
                                                  for t in ts]))
        self.torch.cuda.current_stream(self.device).synchronize()  # the inputs may be temporaries
        return self

    def step(self, n=1):
        self._c(self.lib.lbpf_sp_step(self._h, int(n)))
        return self

    def read(self, field, out=None):
        t = out if out is not None else self.torch.empty((self.ny, self.nx), dtype=self.torch.float32,
                                                          device=self.device)
        self._c(self.lib.lbpf_sp_read(self._h, SP_FIELDS[field], ctypes.c_void_p(t.data_ptr())))
        return t

    def sums(self):
        out = (ctypes.c_double * 3)()
        self._c(self.lib.lbpf_sp_sums(self._h, out))
        return dict(rho_tilde=out[0], mom_x=out[1], mom_y=out[2])

    @property
    def step_count(self):
        return int(self.lib.lbpf_sp_step_count(self._h))


# ---- three-dimensional solver (D3Q15) ------------------------------------------------------

class Params3D(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("pscheme", ctypes.c_int32), ("fsurf", ctypes.c_int32),
                ("visc", ctypes.c_int32), ("bc", ctypes.c_int32), ("clamp_props", ctypes.c_int32),
                ("pad", ctypes.c_int32)] + \
               [(k, ctypes.c_double) for k in ("rho_A", "rho_B", "nu_A", "nu_B", "sigma", "W",
                                               "M_phi", "tau_h", "force_x", "force_y", "force_z",
                                               "gravity")]


FIELDS3D = {"phi": 0, "rho": 1, "ux": 2, "uy": 3, "uz": 4, "p": 5, "mu": 6}
BCS3D = {"periodic": 0, "walls_z": 1}
_P3 = ctypes.POINTER(Params3D)
_I32P = ctypes.POINTER(ctypes.c_int32)
SIGNATURES.update({
    "lbpf3d_workspace_size": (_S, [_P3, ctypes.POINTER(ctypes.c_size_t)]),
    "lbpf3d_create": (_S, [_P3, _V, ctypes.c_size_t, _V, ctypes.POINTER(_V)]),
    "lbpf3d_init": (_S, [_V, _V, _V, _V, _V, _V]),
    "lbpf3d_step": (_S, [_V, ctypes.c_int64]),
    "lbpf3d_read": (_S, [_V, ctypes.c_int32, _V]),
    "lbpf3d_diagnostics": (_S, [_V, ctypes.POINTER(Diag)]),
    "lbpf3d_laplace_dp": (_S, [_V, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.POINTER(ctypes.c_double)]),
    "lbpf3d_shape_count": (ctypes.c_int32, []),
    "lbpf3d_shape_info": (_S, [ctypes.c_int32, _I32P, _I32P, _I32P]),
    "lbpf3d_set_shape": (_S, [_V, ctypes.c_int32]),
    "lbpf3d_get_shape": (ctypes.c_int32, [_V]),
    "lbpf3d_autotune": (_S, [_V, ctypes.c_int32, _V, _I32P]),
    "lbpf3d_state_size": (_S, [_V, ctypes.POINTER(ctypes.c_size_t)]),
    "lbpf3d_save_state": (_S, [_V, _V]),
    "lbpf3d_load_state": (_S, [_V, _V]),
    "lbpf3d_step_count": (ctypes.c_int64, [_V]),
    "lbpf3d_destroy": (_S, [_V]),
    "lbpf3d_last_error": (ctypes.c_char_p, [_V]),
})


def make_params3d(cfg):
    p = Params3D()
    p.nx, p.ny, p.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg["nz"])
    p.variant = VARIANTS[cfg.get("variant", "qim")]
    p.pscheme = PSCHEMES[cfg.get("pscheme", "eq28")]
    p.fsurf = FSURF[cfg.get("fsurf", "mu_grad_phi")]
    p.visc = VISC[cfg.get("visc", "inverse_linear")]
    p.bc = BCS3D[cfg.get("bc", "periodic")]
    p.clamp_props = int(bool(cfg.get("clamp_props", False)))
    for k in ("rho_A", "rho_B", "nu_A", "nu_B", "sigma", "W", "M_phi", "tau_h"):
        setattr(p, k, float(cfg[k]))
    for k in ("force_x", "force_y", "force_z", "gravity"):
        setattr(p, k, float(cfg.get(k, 0.0)))
    return p


def shapes3d():
    lib = library()
    out = []
    for s in range(lib.lbpf3d_shape_count()):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        lib.lbpf3d_shape_info(s, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        out.append((a.value, b.value, c.value))
    return out


class Simulation3D:
    """One D3Q15 two-phase simulation on one GPU: init fields [nz, ny, nx], step N, read fields,
    FP64 diagnostics."""

    def __init__(self, cfg, device="cuda"):
        import torch
        self.torch = torch
        self.lib = library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lbpf solver runs only on the GPU")
        self.device = torch.device(device)
        self.cfg = dict(cfg)
        self.params = make_params3d(cfg)
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        nb = ctypes.c_size_t()
        st = self.lib.lbpf3d_workspace_size(ctypes.byref(self.params), ctypes.byref(nb))
        if st != 0:
            raise LbpfError(st, (self.lib.lbpf3d_last_error(None) or b"").decode())
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        h = ctypes.c_void_p()
        st = self.lib.lbpf3d_create(ctypes.byref(self.params), ctypes.c_void_p(self.workspace.data_ptr()),
                                    ctypes.c_size_t(nb.value), ctypes.c_void_p(stream), ctypes.byref(h))
        if st != 0:
            raise LbpfError(st, (self.lib.lbpf3d_last_error(None) or b"").decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.lbpf3d_destroy(h)
            self._h = None

    def _c(self, st):
        if st != 0:
            raise LbpfError(st, (self.lib.lbpf3d_last_error(self._h) or b"").decode())

    def _as_field(self, a):
        if a is None:
            return None
        t = self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device).contiguous()
        if tuple(t.shape) != self.shape:
            raise ValueError(f"field shape {tuple(t.shape)} != {self.shape}")
        return t

    def init(self, phi, ux=None, uy=None, uz=None, p=None):
        ts = [self._as_field(a) for a in (phi, ux, uy, uz, p)]
        self._c(self.lib.lbpf3d_init(self._h, *[ctypes.c_void_p(t.data_ptr()) if t is not None else None
                                                 for t in ts]))
        self.torch.cuda.current_stream(self.device).synchronize()  # the inputs may be temporaries
        return self

    def step(self, n=1):
        self._c(self.lib.lbpf3d_step(self._h, int(n)))
        return self

    def read(self, field, out=None):
        t = out if out is not None else self.torch.empty(self.shape, dtype=self.torch.float32,
                                                          device=self.device)
        if tuple(t.shape) != self.shape or t.dtype != self.torch.float32 or not t.is_contiguous():
            raise ValueError("output must be a contiguous float32 tensor of the grid's shape")
        self._c(self.lib.lbpf3d_read(self._h, FIELDS3D[field], ctypes.c_void_p(t.data_ptr())))
        return t

    def diagnostics(self, check=True):
        d = Diag()
        st = self.lib.lbpf3d_diagnostics(self._h, ctypes.byref(d))
        if check:
            self._c(st)
        return dict(sum_phi=d.sum_phi, sum_rho=d.sum_rho, max_u=d.max_u, nonfinite=d.nonfinite,
                    step=d.step, status=st)

    def laplace_dp(self, xc, yc, zc, R):
        v = ctypes.c_double()
        self._c(self.lib.lbpf3d_laplace_dp(self._h, float(xc), float(yc), float(zc), float(R), ctypes.byref(v)))
        return v.value

    def set_shape(self, s):
        self._c(self.lib.lbpf3d_set_shape(self._h, int(s)))
        return self

    @property
    def launch_shape(self):
        return int(self.lib.lbpf3d_get_shape(self._h))

    def autotune(self, trial_steps=5, restore=True):
        """Time every launch shape and keep the fastest; with restore the state and step count
        are put back afterwards (through a checkpoint buffer), else they advance."""
        best = ctypes.c_int32()
        scratch = self.torch.empty(self.state_size(), dtype=self.torch.uint8, device=self.device) if restore else None
        ptr = ctypes.c_void_p(scratch.data_ptr()) if restore else None
        self._c(self.lib.lbpf3d_autotune(self._h, int(trial_steps), ptr, ctypes.byref(best)))
        return best.value

    def state_size(self):
        n = ctypes.c_size_t()
        self._c(self.lib.lbpf3d_state_size(self._h, ctypes.byref(n)))
        return n.value

    def save_state(self, out=None):
        buf = out if out is not None else self.torch.empty(self.state_size(), dtype=self.torch.uint8,
                                                           device=self.device)
        self._c(self.lib.lbpf3d_save_state(self._h, ctypes.c_void_p(buf.data_ptr())))
        return buf

    def load_state(self, buf):
        if buf.numel() < self.state_size() or not buf.is_cuda:
            raise ValueError("checkpoint buffer too small or not on the GPU")
        self._c(self.lib.lbpf3d_load_state(self._h, ctypes.c_void_p(buf.data_ptr())))
        return self

    @property
    def step_count(self):
        return int(self.lib.lbpf3d_step_count(self._h))
