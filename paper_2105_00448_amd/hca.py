"""ctypes binding of libhca (include/hca.h): argument marshalling only.

Every computation runs in the HIP library.  If libhca.so is missing or
cannot be loaded this module raises; there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhca.so")
_lib = None

OK, E_INVALID, E_NOMEM, E_DEVICE, E_NOCONV, E_NONFINITE, E_SINGULAR, E_RANGE = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "HCA_OK", -1: "HCA_E_INVALID", -2: "HCA_E_NOMEM", -3: "HCA_E_DEVICE",
                -4: "HCA_E_NOCONV", -5: "HCA_E_NONFINITE", -6: "HCA_E_SINGULAR", -7: "HCA_E_RANGE"}

F_O2, F_DRUG1, F_DRUG2, F_CELL, F_P53, F_VEGF_IC, F_PHI, F_VESSEL_W, F_VEGF, F_DRUG3 = range(10)
FIELDS = {"K": F_O2, "G1": F_DRUG1, "G2": F_DRUG2, "L": F_CELL, "P": F_P53, "Vc": F_VEGF_IC,
          "phi": F_PHI, "w": F_VESSEL_W, "V": F_VEGF, "G3": F_DRUG3}

PH_O2, PH_DRUGS, PH_ODE, PH_CA, PH_STATS, PH_ADVANCE, PH_VEGF = 1, 2, 4, 8, 16, 32, 64
PH_ALL = 127
MAX_DOSES = 64


class Params(C.Structure):
    _fields_ = [
        ("h_um", C.c_double), ("dt_min", C.c_double),
        ("D_K", C.c_double), ("r_k", C.c_double), ("K0", C.c_double), ("phi_K", C.c_double),
        ("K1", C.c_double),
        ("D_G", C.c_double), ("psi_G", C.c_double), ("kappa_G", C.c_double),
        ("k_pk", C.c_double * 2), ("G_ref", C.c_double * 2), ("b_int", C.c_int32 * 2),
        ("k1", C.c_double), ("k1p", C.c_double), ("K_p53", C.c_double), ("k2", C.c_double),
        ("k2p", C.c_double), ("k2pp", C.c_double), ("J5", C.c_double), ("K_V", C.c_double),
        ("K_phi", C.c_double), ("T_cycle", C.c_double),
        ("ode_substeps", C.c_int32),
        ("precond", C.c_int32), ("cg_rtol", C.c_double), ("cg_maxit", C.c_int32),
        ("mg_smooth", C.c_int32), ("mg_coarse_max", C.c_int32),
        ("init_rtol", C.c_double), ("init_maxit", C.c_int32), ("profile", C.c_int32),
        ("graphs", C.c_int32), ("autotune", C.c_int32),
        ("pde_substeps", C.c_int32), ("pde_theta", C.c_double), ("o2_newton", C.c_int32),
        ("pk_mm", C.c_int32), ("mm_vmax", C.c_double), ("mm_km", C.c_double),
        ("vegf", C.c_int32), ("D_V", C.c_double), ("psi_V", C.c_double), ("sec_V", C.c_double),
        ("dv_min", C.c_double), ("V_low", C.c_double), ("V_high", C.c_double),
        ("p_death", C.c_double), ("birth_per_V", C.c_double), ("w_new", C.c_double),
        ("drug3", C.c_int32), ("epi_w1", C.c_double), ("epi_w2", C.c_double), ("epi_w3", C.c_double),
        ("epi_q2", C.c_double), ("epi_q3", C.c_double), ("epi_cl", C.c_double),
        ("G_ref3", C.c_double), ("b_int3", C.c_int32),
        ("x0_extrapolate", C.c_int32),
        ("precision", C.c_int32),
        ("mg_fuse", C.c_int32),
    ]


class Replicate(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("seed", C.c_uint64),
        ("cell", C.POINTER(C.c_uint8)), ("vessel_w", C.POINTER(C.c_double)),
        ("n_doses", C.c_int32 * 2),
        ("dose_t_min", C.POINTER(C.c_double) * 2), ("dose_amt", C.POINTER(C.c_double) * 2),
        ("n_doses3", C.c_int32), ("dose_t_min3", C.POINTER(C.c_double)),
        ("dose_amt3", C.POINTER(C.c_double)),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("n_cancer", C.c_int64), ("n_stroma", C.c_int64),
        ("n_empty", C.c_int64), ("n_vessel", C.c_int64),
        ("committed", C.c_int64), ("divisions", C.c_int64), ("kills", C.c_int64),
        ("nospace", C.c_int64), ("lost", C.c_int64),
        ("total_divisions", C.c_int64), ("total_kills", C.c_int64),
        ("cg_iters", C.c_int32 * 3), ("cg_relres", C.c_double * 3),
        ("nonfinite", C.c_int32), ("init_picard_iters", C.c_int32),
        ("sur_voxels", C.c_int64), ("sur_fallbacks", C.c_int64),
        ("cg_iters_vegf", C.c_int32), ("cg_relres_vegf", C.c_double),
        ("vessel_births", C.c_int64), ("vessel_deaths", C.c_int64),
        ("total_births", C.c_int64), ("total_deaths", C.c_int64),
        ("cg_iters_drug3", C.c_int32), ("cg_relres_drug3", C.c_double),
    ]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if hasattr(v, "__len__") else v
        return d


MLP_NIN, MLP_NHID, MLP_NOUT, MLP_NPARAM = 6, 64, 3, 8963


class Mlp(C.Structure):
    _fields_ = [
        ("theta", C.c_void_p), ("theta_is_device", C.c_int32),
        ("in_mean", C.c_float * MLP_NIN), ("in_scale", C.c_float * MLP_NIN),
        ("out_mean", C.c_float * MLP_NOUT), ("out_scale", C.c_float * MLP_NOUT),
        ("in_lo", C.c_float * MLP_NIN), ("in_hi", C.c_float * MLP_NIN),
        ("box_check", C.c_int32),
    ]

    def stats(self):
        return {k: np.array(getattr(self, k), dtype=np.float32)
                for k in ("in_mean", "in_scale", "out_mean", "out_scale", "in_lo", "in_hi")}


def lib():
    """Load libhca.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built: run `python -m paper_2105_00448_amd.build`")
    L = C.CDLL(_LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    sigs = {
        "hca_default_params": (C.c_int, [P(Params)]),
        "hca_init": (C.c_int, [P(vp), P(Params), P(Replicate), C.c_int, vp]),
        "hca_step": (C.c_int, [vp, C.c_int]),
        "hca_run_phases": (C.c_int, [vp, C.c_uint]),
        "hca_fields": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_size_t, C.c_int]),
        "hca_set_field": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_size_t, C.c_int]),
        "hca_set_step": (C.c_int, [vp, C.c_int64]),
        "hca_state_bytes": (C.c_int, [vp, C.c_int, P(C.c_size_t)]),
        "hca_export_state": (C.c_int, [vp, C.c_int, vp, C.c_size_t, C.c_int]),
        "hca_import_state": (C.c_int, [vp, C.c_int, vp, C.c_size_t, C.c_int]),
        "hca_init_from_state": (C.c_int, [P(vp), P(Params), P(Replicate), P(vp), P(C.c_size_t),
                                          C.c_int, vp]),
        "hca_stats": (C.c_int, [vp, C.c_int, P(Stats)]),
        "hca_kernel_time": (C.c_int, [vp, C.c_int, P(C.c_double), P(C.c_int64), P(C.c_double)]),
        "hca_kernel_name": (C.c_char_p, [C.c_int]),
        "hca_num_kernels": (C.c_int, []),
        "hca_reset_kernel_time": (C.c_int, [vp]),
        "hca_set_profile": (C.c_int, [vp, C.c_int]),
        "hca_synchronize": (C.c_int, [vp]),
        "hca_last_error": (C.c_char_p, [vp]),
        "hca_destroy": (None, [vp]),
        "hca_set_surrogate": (C.c_int, [vp, P(Mlp), C.c_double]),
        "hca_tile_shape": (C.c_int, [vp, C.c_int, P(C.c_int32), P(C.c_int32), P(C.c_int32)]),
        "hca_harvest_step": (C.c_int, [vp, vp, vp, C.c_int64, P(C.c_int64)]),
        "hca_mlp_trainer_create": (C.c_int, [P(vp), vp, vp, C.c_int64, C.c_uint64, vp]),
        "hca_mlp_trainer_set_params": (C.c_int, [vp, vp, C.c_int]),
        "hca_mlp_trainer_params": (C.c_int, [vp, vp, C.c_int]),
        "hca_mlp_trainer_data": (C.c_int, [vp, vp, vp]),
        "hca_mlp_trainer_export": (C.c_int, [vp, P(Mlp)]),
        "hca_mlp_gradient": (C.c_int, [vp, vp, C.c_int, vp, P(C.c_float)]),
        "hca_mlp_train": (C.c_int, [vp, C.c_int, C.c_int, C.c_float, vp]),
        "hca_mlp_eval": (C.c_int, [vp, vp, C.c_int64, C.c_int, vp]),
        "hca_mlp_apply_gradient": (C.c_int, [vp, vp, C.c_int, C.c_float]),
        "hca_mlp_gradient_noalloc": (C.c_int, [vp, vp, vp, C.c_int64, vp, C.c_int, vp, vp, vp]),
        "hca_mlp_trainer_last_error": (C.c_char_p, [vp]),
        "hca_mlp_trainer_destroy": (None, [vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class HcaError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")


def default_params(**overrides):
    p = Params()
    st = lib().hca_default_params(C.byref(p))
    if st != OK:
        raise HcaError(st, "hca_default_params")
    for k, v in overrides.items():
        if isinstance(v, (tuple, list)):
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(p, k, v)
    return p


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Simulation:
    """One context: a batch of replicates stepped together.

    ``replicates``: list of (cell uint8 (nz,ny,nx), w float64 (nz,ny,nx), seed,
    (dose_times, dose_amts) per drug as a pair of sequences; a third entry in
    each is the third drug's schedule).
    """

    def __init__(self, replicates, params=None, stream=None, states=None):
        """``states``: optional list of state blobs (uint8 numpy arrays from
        ``export_state``), one per replicate: the context then resumes from
        them (hca_init_from_state) and each replicate's cell and w may be
        None, its shape taken from the blob."""
        self._lib = lib()
        self.params = params if params is not None else default_params()
        self.shapes = []
        keep = []
        reps = (Replicate * len(replicates))()
        for r, (cell, w, seed, sched) in enumerate(replicates):
            R = reps[r]
            if states is not None and cell is None:
                hdr = np.frombuffer(states[r][:32].tobytes(), dtype=np.int32)
                nx, ny, nz = int(hdr[4]), int(hdr[5]), int(hdr[6])
            else:
                cell = np.ascontiguousarray(cell, dtype=np.uint8)
                w = np.ascontiguousarray(w, dtype=np.float64)
                if cell.shape != w.shape or cell.ndim != 3:
                    raise ValueError("cell and w must be (nz, ny, nx) arrays of one shape")
                nz, ny, nx = cell.shape
                R.cell = cell.ctypes.data_as(C.POINTER(C.c_uint8))
                R.vessel_w = _dptr(w)
                keep += [cell, w]
            self.shapes.append((nz, ny, nx))
            R.nx, R.ny, R.nz, R.seed = nx, ny, nz, int(seed)
            times, amts = sched
            for d in range(2):
                t = np.ascontiguousarray(times[d], dtype=np.float64)
                a = np.ascontiguousarray(amts[d], dtype=np.float64)
                R.n_doses[d] = len(t)
                R.dose_t_min[d] = _dptr(t)
                R.dose_amt[d] = _dptr(a)
                keep += [t, a]
            if len(times) > 2:
                t = np.ascontiguousarray(times[2], dtype=np.float64)
                a = np.ascontiguousarray(amts[2], dtype=np.float64)
                R.n_doses3 = len(t)
                R.dose_t_min3 = _dptr(t)
                R.dose_amt3 = _dptr(a)
                keep += [t, a]
        h = C.c_void_p()
        if states is None:
            st = self._lib.hca_init(C.byref(h), C.byref(self.params), reps, len(replicates),
                                    C.c_void_p(stream) if stream else None)
        else:
            blobs = [np.ascontiguousarray(b, dtype=np.uint8) for b in states]
            keep += blobs
            ptrs = (C.c_void_p * len(blobs))(*[b.ctypes.data for b in blobs])
            sizes = (C.c_size_t * len(blobs))(*[b.nbytes for b in blobs])
            st = self._lib.hca_init_from_state(C.byref(h), C.byref(self.params), reps, ptrs, sizes,
                                               len(replicates), C.c_void_p(stream) if stream else None)
        if st != OK:
            raise HcaError(st, "hca_init failed (details on stderr)")
        self._h = h

    # -- stepping --------------------------------------------------------
    def _check(self, st, what):
        if st != OK:
            raise HcaError(st, f"{what}: {self._lib.hca_last_error(self._h).decode()}")

    def step(self, n=1):
        self._check(self._lib.hca_step(self._h, n), "hca_step")

    def run_phases(self, mask):
        self._check(self._lib.hca_run_phases(self._h, mask), "hca_run_phases")

    def set_step(self, n):
        self._check(self._lib.hca_set_step(self._h, n), "hca_set_step")

    # -- state -----------------------------------------------------------
    def _check_rep(self, rep, f):
        if not 0 <= rep < len(self.shapes):
            # let the library report the range error
            dummy = np.empty(1, dtype=np.uint8)
            self._check(self._lib.hca_fields(self._h, rep, f, dummy.ctypes.data, 0, 0),
                        "hca_fields")

    def field(self, name, rep=0):
        f = FIELDS[name]
        self._check_rep(rep, f)
        shape = self.shapes[rep]
        out = np.empty(shape, dtype=np.uint8 if f == F_CELL else np.float64)
        self._check(self._lib.hca_fields(self._h, rep, f, out.ctypes.data, out.nbytes, 0),
                    "hca_fields")
        return out

    def field_to_device(self, name, tensor, rep=0):
        """Copy into a caller-owned torch device tensor (device-to-device)."""
        f = FIELDS[name]
        self._check(self._lib.hca_fields(self._h, rep, f, tensor.data_ptr(),
                                         tensor.numel() * tensor.element_size(), 1), "hca_fields")
        return tensor

    def set_field(self, name, arr, rep=0):
        f = FIELDS[name]
        a = np.ascontiguousarray(arr, dtype=np.uint8 if f == F_CELL else np.float64)
        self._check(self._lib.hca_set_field(self._h, rep, f, a.ctypes.data, a.nbytes, 0),
                    "hca_set_field")

    def state_bytes(self, rep=0):
        n = C.c_size_t()
        self._check(self._lib.hca_state_bytes(self._h, rep, C.byref(n)), "hca_state_bytes")
        return n.value

    def export_state(self, rep=0):
        """The replicate's complete state (hca_export_state) as a uint8 array."""
        out = np.empty(self.state_bytes(rep), dtype=np.uint8)
        self._check(self._lib.hca_export_state(self._h, rep, out.ctypes.data, out.nbytes, 0),
                    "hca_export_state")
        return out

    def import_state(self, blob, rep=0):
        b = np.ascontiguousarray(blob, dtype=np.uint8)
        self._check(self._lib.hca_import_state(self._h, rep, b.ctypes.data, b.nbytes, 0),
                    "hca_import_state")

    def tile_shape(self, rep=0):
        tx, ty, tz = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self._lib.hca_tile_shape(self._h, rep, C.byref(tx), C.byref(ty), C.byref(tz)),
                    "hca_tile_shape")
        return tx.value, ty.value, tz.value

    def set_field_from_device(self, name, tensor, rep=0):
        """Overwrite a state field from a torch device tensor (device-to-device)."""
        f = FIELDS[name]
        self._check(self._lib.hca_set_field(self._h, rep, f, tensor.data_ptr(),
                                            tensor.numel() * tensor.element_size(), 1),
                    "hca_set_field")

    def stats(self, rep=0):
        s = Stats()
        self._check(self._lib.hca_stats(self._h, rep, C.byref(s)), "hca_stats")
        return s.as_dict()

    def kernel_times(self):
        out = {}
        for k in range(self._lib.hca_num_kernels()):
            ms, n, b = C.c_double(), C.c_int64(), C.c_double()
            self._check(self._lib.hca_kernel_time(self._h, k, C.byref(ms), C.byref(n), C.byref(b)),
                        "hca_kernel_time")
            out[self._lib.hca_kernel_name(k).decode()] = dict(ms=ms.value, launches=n.value,
                                                              bytes_per_launch=b.value)
        return out

    def set_profile(self, profile):
        self._check(self._lib.hca_set_profile(self._h, int(profile)), "hca_set_profile")

    def reset_kernel_times(self):
        self._check(self._lib.hca_reset_kernel_time(self._h), "hca_reset_kernel_time")

    def synchronize(self):
        self._check(self._lib.hca_synchronize(self._h), "hca_synchronize")

    # -- surrogate ---------------------------------------------------------
    def set_surrogate(self, net, margin=1e-3):
        """net: an Mlp (e.g. Trainer.export()) or None for the plain integrator."""
        self._check(self._lib.hca_set_surrogate(self._h, C.byref(net) if net is not None else None,
                                                float(margin)), "hca_set_surrogate")

    def harvest_step(self, X, Y):
        """One coupled step that writes training rows into the device tensors
        X (cap x 6) and Y (cap x 3), float32; returns the rows written."""
        n = C.c_int64()
        self._check(self._lib.hca_harvest_step(self._h, X.data_ptr(), Y.data_ptr(),
                                               min(X.shape[0], Y.shape[0]), C.byref(n)),
                    "hca_harvest_step")
        return n.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hca_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def mlp_gradient_noalloc(theta, Xs, Ys, idx, grad, loss=None, stream=None):
    """hca_mlp_gradient_noalloc on device tensors (theta, Xs, Ys float32;
    idx int32; grad float32 NPARAM; loss a one-element float32 tensor or
    None); enqueues only."""
    st = lib().hca_mlp_gradient_noalloc(theta.data_ptr(), Xs.data_ptr(), Ys.data_ptr(),
                                        Xs.shape[0], idx.data_ptr(), idx.numel(), grad.data_ptr(),
                                        loss.data_ptr() if loss is not None else None,
                                        C.c_void_p(stream) if stream else None)
    if st != OK:
        raise HcaError(st, "hca_mlp_gradient_noalloc")


def schedule_tuple(sched):
    """(times, amts) pair from a synth.DoseSchedule-like object."""
    return (tuple(tuple(t) for t in sched.times), tuple(tuple(a) for a in sched.amts))


class Trainer:
    """hca_mlp_trainer: X (n x 6) and Y (n x 3) are float32 device tensors."""

    def __init__(self, X, Y, seed=0, stream=None):
        self._lib = lib()
        if X.shape[0] != Y.shape[0] or X.shape[1:] != (MLP_NIN,) or Y.shape[1:] != (MLP_NOUT,):
            raise ValueError("X must be (n, 6) and Y (n, 3)")
        self.n = X.shape[0]
        h = C.c_void_p()
        st = self._lib.hca_mlp_trainer_create(C.byref(h), X.data_ptr(), Y.data_ptr(), self.n,
                                              int(seed), C.c_void_p(stream) if stream else None)
        if st != OK:
            raise HcaError(st, "hca_mlp_trainer_create failed (details on stderr)")
        self._h = h

    def _check(self, st, what):
        if st != OK:
            raise HcaError(st, f"{what}: {self._lib.hca_mlp_trainer_last_error(self._h).decode()}")

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        if a.shape != (MLP_NPARAM,):
            raise ValueError("theta must have HCA_MLP_NPARAM values")
        self._check(self._lib.hca_mlp_trainer_set_params(self._h, a.ctypes.data, 0), "set_params")

    def params(self):
        a = np.empty(MLP_NPARAM, dtype=np.float32)
        self._check(self._lib.hca_mlp_trainer_params(self._h, a.ctypes.data, 0), "params")
        return a

    def data(self, Xs, Ys):
        self._check(self._lib.hca_mlp_trainer_data(self._h, Xs.data_ptr(), Ys.data_ptr()), "data")

    def export(self):
        m = Mlp()
        self._check(self._lib.hca_mlp_trainer_export(self._h, C.byref(m)), "export")
        return m

    def gradient(self, idx, grad):
        """idx: int32 device tensor (batch); grad: float32 device tensor (NPARAM)."""
        loss = C.c_float()
        self._check(self._lib.hca_mlp_gradient(self._h, idx.data_ptr(), idx.numel(),
                                               grad.data_ptr(), C.byref(loss)), "gradient")
        return loss.value

    def train(self, steps, batch=1024, lr=1e-3):
        out = np.empty(steps, dtype=np.float32)
        self._check(self._lib.hca_mlp_train(self._h, steps, batch, float(lr), out.ctypes.data),
                    "train")
        return out

    def apply_gradient(self, grad, lr):
        """One Adam step from a gradient (numpy float32 array on the host, or
        a float32 device tensor)."""
        if isinstance(grad, np.ndarray):
            a = np.ascontiguousarray(grad, dtype=np.float32)
            if a.shape != (MLP_NPARAM,):
                raise ValueError("grad must have HCA_MLP_NPARAM values")
            st = self._lib.hca_mlp_apply_gradient(self._h, a.ctypes.data, 0, float(lr))
        else:
            st = self._lib.hca_mlp_apply_gradient(self._h, grad.data_ptr(), 1, float(lr))
        self._check(st, "apply_gradient")

    def eval(self, X, Y, raw=True):
        self._check(self._lib.hca_mlp_eval(self._h, X.data_ptr(), X.shape[0], 1 if raw else 0,
                                           Y.data_ptr()), "eval")
        return Y

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hca_mlp_trainer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
