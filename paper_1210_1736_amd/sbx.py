"""ctypes binding of libsbx (the C ABI declared in include/sbx.h).

Argument marshalling only: every step of the field solve runs in the HIP
kernels of the library.  Importing this module loads libsbx.so and raises if
it is missing; there is no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsbx.so")

SBX_OK, SBX_EINVAL, SBX_ENOMEM, SBX_EDEVICE, SBX_EQCRIT, SBX_ESTATE, SBX_EPARITY = 0, -1, -2, -3, -4, -5, -6
SBX_FP32, SBX_FP64 = 0, 1
SBX_CENTRE_FIXED, SBX_CENTRE_COM, SBX_CENTRE_DENSITY = 0, 1, 2
CORE, RING, OUTER, LOST = 0, 1, 2, 3

N_PHASES = 11
PHASES = ["start", "zero", "pre", "deposit", "fwd_x", "fwd_y", "zpass", "inv_y", "inv_x", "force",
          "sort"]

_NAMES = {0: "SBX_OK", -1: "SBX_EINVAL", -2: "SBX_ENOMEM", -3: "SBX_EDEVICE", -4: "SBX_EQCRIT",
          -5: "SBX_ESTATE", -6: "SBX_EPARITY"}


class SbxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class sbx_level(C.Structure):
    _fields_ = [("n", C.c_int32), ("R", C.c_double), ("q", C.c_double)]


class sbx_hierarchy(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("lv", sbx_level * 3), ("centring", C.c_int32),
                ("centre", C.c_double * 3), ("outer_centre", C.c_double * 3)]


class sbx_config(C.Structure):
    _fields_ = [("prec", C.c_int32), ("G", C.c_double), ("h0_mode", C.c_int32),
                ("taylor", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p)]


class sbx_diag(C.Structure):
    _fields_ = [("ekin", C.c_double * 8), ("epot", C.c_double * 8), ("L", (C.c_double * 3) * 8),
                ("disc_sigR", C.c_double), ("disc_sigz", C.c_double), ("n_lost", C.c_int64),
                ("n_live", C.c_int64 * 8)]

    def as_dict(self):
        return {"ekin": np.array(self.ekin[:]), "epot": np.array(self.epot[:]),
                "L": np.array([self.L[i][:] for i in range(8)]), "disc_sigR": self.disc_sigR,
                "disc_sigz": self.disc_sigz, "n_lost": int(self.n_lost),
                "n_live": np.array(self.n_live[:])}


class sbx_disc_query(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("annulus", C.c_double * 2), ("n_z", C.c_int32),
                ("z_max", C.c_double), ("comp", C.c_int32), ("galaxy", C.c_int32)]


class sbx_disc_result(C.Structure):
    _fields_ = [("e_heat", C.c_double), ("sig_R", C.c_double), ("sig_phi", C.c_double),
                ("sig_z", C.c_double), ("sig_tot2", C.c_double), ("bulk_v", C.c_double * 3),
                ("n_disc", C.c_int64), ("n_annulus", C.c_int64)]


def _load():
    # PyTorch wheels carry their own copy of the HIP runtime under the same
    # soname; loading torch first makes the library bind to that one copy, so
    # torch tensors and streams and this library share one runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1210_1736_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, S = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_int
    dp = C.POINTER(C.c_double)
    sig = {
        "sbx_last_error": (C.c_char_p, []),
        "sbx_validate_hierarchies": (S, [I32, C.POINTER(sbx_hierarchy)]),
        "sbx_q_crit": (D, [I32, D, D, D]),
        "sbx_create": (S, [C.POINTER(sbx_config), C.POINTER(P)]),
        "sbx_destroy": (None, [P]),
        "sbx_load_particles": (S, [P, I64, P, P, P, P, P]),
        "sbx_build_grids": (S, [P, I32, C.POINTER(sbx_hierarchy)]),
        "sbx_compute_forces": (S, [P, P, P]),
        "sbx_step": (S, [P, D, I32, I32]),
        "sbx_get_particles": (S, [P, P, P, P]),
        "sbx_get_centres": (S, [P, P]),
        "sbx_get_indices": (S, [P, I32, I32, P, P]),
        "sbx_get_grid": (S, [P, I32, I32, I32, P]),
        "sbx_diagnostics": (S, [P, D, C.POINTER(sbx_diag)]),
        "sbx_diag_log": (S, [P, I32, C.POINTER(sbx_diag), C.POINTER(I32)]),
        "sbx_sync": (S, [P]),
        "sbx_set_sort_interval": (S, [P, I32]),
        "sbx_set_outer_merge": (S, [P, I32]),
        "sbx_set_deterministic_deposit": (S, [P, I32]),
        "sbx_adjoint_segment": (S, [P, D, I32, I32, I32, I32, P, P, P, P]),
        "sbx_adjoint_segment_device": (S, [P, D, I32, I32, I32, I32, P, P, P, P]),
        "sbx_load_particles_device": (S, [P, I64, P, P, P, P, P]),
        "sbx_disc_analysis": (S, [P, P, P, P, P, P, P]),
        "sbx_disc_modes": (S, [P, I32, I32, I32, D, I32, P]),
        "sbx_get_particles_device": (S, [P, P, P, P]),
        "sbx_bind_device_particles": (S, [P, I64, P, P, P, P, P, P]),
        "sbx_save": (S, [P, C.c_char_p]),
        "sbx_get_counts": (S, [P, C.POINTER(I64), C.POINTER(I32)]),
        "sbx_load": (S, [P, C.c_char_p]),
        "sbx_count_live": (S, [P, C.POINTER(I64)]),
        "sbx_profile_begin": (S, [P, I32]),
        "sbx_profile_end": (S, [P, I32, P, P]),
        "sbx_batch_create": (S, [C.POINTER(P), I32, P, C.POINTER(P)]),
        "sbx_batch_step": (S, [P, P, I32]),
        "sbx_batch_sync": (S, [P]),
        "sbx_batch_set_sort_interval": (S, [P, I32]),
        "sbx_batch_destroy": (None, [P]),
        "sbx_poisson_create": (S, [I32, D, D, D, I32, I32, I32, P, C.POINTER(P)]),
        "sbx_poisson_destroy": (None, [P]),
        "sbx_poisson_solve": (S, [P, I32, P, P]),
        "sbx_poisson_solve_noalloc": (S, [P, I32, P, P]),
        "sbx_poisson_green": (S, [P, P, dp]),
        "sbx_poisson_bytes": (I64, [P]),
        "sbx_set_fft_schedule": (S, [I32]),
        "sbx_set_plane_threads": (S, [I32]),
        "sbx_set_fft_form": (S, [I32]),
        "sbx_fft_tuning_report": (I64, [C.c_char_p, I64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def last_error() -> str:
    return _lib.sbx_last_error().decode()


def _check(status):
    if status != SBX_OK:
        raise SbxError(status, last_error())


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_hierarchy(levels, centring=SBX_CENTRE_FIXED, centre=(0.0, 0.0, 0.0),
                   outer_centre=(0.0, 0.0, 0.0)) -> sbx_hierarchy:
    """levels: [(n, R, q)] with 1 or 3 entries (inner, middle, outer)."""
    h = sbx_hierarchy()
    h.n_levels = len(levels)
    for i, (n, R, q) in enumerate(levels):
        h.lv[i] = sbx_level(int(n), float(R), float(q))
    h.centring = int(centring)
    h.centre[:] = [float(c) for c in centre]
    h.outer_centre[:] = [float(c) for c in outer_centre]
    return h


def hierarchy_array(hs):
    arr = (sbx_hierarchy * len(hs))()
    for i, h in enumerate(hs):
        arr[i] = h
    return arr


def sbx_validate_hierarchies(hs) -> int:
    arr = hierarchy_array(hs)
    return _lib.sbx_validate_hierarchies(len(hs), arr)


def sbx_q_crit(n, R_core, R_out, R_sys) -> float:
    return _lib.sbx_q_crit(n, R_core, R_out, R_sys)


def sbx_set_fft_schedule(values_per_thread):
    """Pin the FFT line schedule (16 or 32 values per thread) for plans made
    from now on; 0 lets the launch-shape tuner choose."""
    _check(_lib.sbx_set_fft_schedule(int(values_per_thread)))


def sbx_set_fft_form(form):
    """Pin the form of the solves for plans made from now on: 3 plane-fused
    passes (where a plane fits in LDS), 5 line passes, 0 the tuner's
    choice."""
    _check(_lib.sbx_set_fft_form(int(form)))


def sbx_set_plane_threads(nt):
    """Pin the block size of the plane-fused passes (256, 512 or 1024) for
    plans made from now on; 0 lets the tuner choose."""
    _check(_lib.sbx_set_plane_threads(int(nt)))


def sbx_fft_tuning_report() -> str:
    """The launch shapes (block size, persistent grid, line schedule) the
    tuner has chosen so far, one line per precision, size, count and pass."""
    n = _lib.sbx_fft_tuning_report(None, 0)
    buf = C.create_string_buffer(int(n) + 1)
    _lib.sbx_fft_tuning_report(buf, int(n) + 1)
    return buf.value.decode()


class Context:
    """One sbx_ctx: particles, grids, forces and steps on one device."""

    def __init__(self, prec=SBX_FP32, G=1.0, h0_mode=0, taylor=1, device=0, stream=None):
        cfg = sbx_config(prec, G, h0_mode, taylor, device, stream)
        h = C.c_void_p()
        _check(_lib.sbx_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self.prec = prec
        self.n = 0
        self.ngal = 0
        self.bound_state = None  # storage borrowed by sbx_bind_device_particles, kept alive here

    def close(self):
        if self._h:
            _lib.sbx_destroy(self._h)
            self._h = None
        self.bound_state = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- inputs ---------------------------------------------------------------
    def sbx_load_particles(self, x, v, m, comp, gal):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        m = np.ascontiguousarray(m, dtype=np.float64)
        comp = np.ascontiguousarray(comp, dtype=np.int8)
        gal = np.ascontiguousarray(gal, dtype=np.int8)
        n = m.shape[0]
        if x.shape != (n, 3) or v.shape != (n, 3) or comp.shape != (n,) or gal.shape != (n,):
            raise ValueError("shapes: x, v (n,3); m, comp, gal (n,)")
        _check(_lib.sbx_load_particles(self._h, n, _ptr(x), _ptr(v), _ptr(m), _ptr(comp), _ptr(gal)))
        self.n = n

    def sbx_load_particles_device(self, n, x, v, m, comp, gal):
        """Device pointers (ints, e.g. tensor.data_ptr()): x, v float64 (n,3),
        m float64 (n,), comp, gal int8 (n,), on the context's device."""
        _check(_lib.sbx_load_particles_device(self._h, int(n), C.c_void_p(x), C.c_void_p(v),
                                              C.c_void_p(m), C.c_void_p(comp), C.c_void_p(gal)))
        self.n = int(n)

    def sbx_bind_device_particles(self, n, x, v, m, comp, gal, lost):
        """Borrow device storage (ints, e.g. tensor.data_ptr()): x, v as 3 x n
        arrays and m (n,) in the context precision, comp, gal int8 (n,), lost
        uint8 (n,).  The caller keeps the storage alive while bound."""
        vp = C.c_void_p
        _check(_lib.sbx_bind_device_particles(self._h, int(n), vp(x), vp(v), vp(m), vp(comp),
                                              vp(gal), vp(lost)))
        self.n = int(n)

    def sbx_save(self, path):
        _check(_lib.sbx_save(self._h, os.fsencode(path)))

    def sbx_load(self, path):
        _check(_lib.sbx_load(self._h, os.fsencode(path)))
        n, ng = C.c_int64(), C.c_int32()
        _check(_lib.sbx_get_counts(self._h, C.byref(n), C.byref(ng)))
        self.n, self.ngal = n.value, ng.value

    def sbx_get_particles_device(self, x=None, v=None, lost=None):
        """Device pointers (ints) for x, v float64 (n,3) and lost uint8 (n,)."""
        vp = lambda a: C.c_void_p(a) if a else None
        _check(_lib.sbx_get_particles_device(self._h, vp(x), vp(v), vp(lost)))

    def sbx_adjoint_segment_device(self, dt, nsteps, ckpt_every, sel_comp, sel_gal, grad_m, grad_x,
                                   grad_v):
        """Gradients into device pointers (ints or None); returns the loss."""
        loss = np.zeros(1)
        vp = lambda a: C.c_void_p(a) if a else None
        _check(_lib.sbx_adjoint_segment_device(self._h, float(dt), int(nsteps), int(ckpt_every),
                                               int(sel_comp), int(sel_gal), _ptr(loss), vp(grad_m),
                                               vp(grad_x), vp(grad_v)))
        return float(loss[0])

    def sbx_disc_analysis(self, n_bins, annulus, n_z, z_max, comp=0, galaxy=0):
        """Disc diagnostics (see sbx.h) as a dict."""
        q = sbx_disc_query(int(n_bins), (C.c_double * 2)(*annulus), int(n_z), float(z_max), int(comp),
                           int(galaxy))
        r = sbx_disc_result()
        br, bv, bz, rz = np.empty(n_bins), np.empty(n_bins), np.empty(n_bins), np.empty(n_z)
        _check(_lib.sbx_disc_analysis(self._h, C.byref(q), C.byref(r), _ptr(br), _ptr(bv), _ptr(bz),
                                      _ptr(rz)))
        return {"e_heat": r.e_heat, "sig_R": r.sig_R, "sig_phi": r.sig_phi, "sig_z": r.sig_z,
                "sig_tot2": r.sig_tot2, "bulk_v": np.array(r.bulk_v[:]), "n_disc": r.n_disc,
                "n_annulus": r.n_annulus, "bin_r": br, "bin_vc": bv, "bin_rms_z": bz, "rho_z": rz}

    def sbx_disc_modes(self, n_rbins, r_max, m_max, comp=0, galaxy=0):
        """(n_rbins, m_max + 1) complex Fourier coefficients (see sbx.h)."""
        out = np.empty(n_rbins * (m_max + 1) * 2)
        _check(_lib.sbx_disc_modes(self._h, int(comp), int(galaxy), int(n_rbins), float(r_max),
                                   int(m_max), _ptr(out)))
        return out.view(np.complex128).reshape(n_rbins, m_max + 1)

    def sbx_build_grids(self, hierarchies):
        arr = hierarchy_array(hierarchies)
        _check(_lib.sbx_build_grids(self._h, len(hierarchies), arr))
        self.ngal = len(hierarchies)
        self.hier = list(hierarchies)

    # -- work -----------------------------------------------------------------
    def sbx_compute_forces(self):
        acc = np.empty((self.n, 3))
        pot = np.empty(self.n)
        _check(_lib.sbx_compute_forces(self._h, _ptr(acc), _ptr(pot)))
        return acc, pot

    def sbx_step(self, dt, nsteps=1, diag_every=0):
        _check(_lib.sbx_step(self._h, float(dt), int(nsteps), int(diag_every)))

    def sbx_sync(self):
        _check(_lib.sbx_sync(self._h))

    def sbx_adjoint_segment(self, dt, nsteps, ckpt_every=2, sel_comp=0, sel_gal=0, grads=True):
        """Loss and gradients of a differentiable segment (see sbx.h)."""
        loss = np.zeros(1)
        gm = np.empty(self.n) if grads else None
        gx = np.empty((self.n, 3)) if grads else None
        gv = np.empty((self.n, 3)) if grads else None
        _check(_lib.sbx_adjoint_segment(self._h, float(dt), int(nsteps), int(ckpt_every), int(sel_comp),
                                        int(sel_gal), _ptr(loss), _ptr(gm), _ptr(gx), _ptr(gv)))
        return float(loss[0]), gm, gx, gv

    def sbx_set_outer_merge(self, merge):
        _check(_lib.sbx_set_outer_merge(self._h, int(merge)))

    def sbx_set_deterministic_deposit(self, on):
        """Fixed-point (order-independent, bit-reproducible) mass assignment."""
        _check(_lib.sbx_set_deterministic_deposit(self._h, int(on)))

    def sbx_set_sort_interval(self, every):
        _check(_lib.sbx_set_sort_interval(self._h, int(every)))

    # -- outputs --------------------------------------------------------------
    def sbx_get_particles(self):
        x = np.empty((self.n, 3)); v = np.empty((self.n, 3)); lost = np.empty(self.n, np.uint8)
        _check(_lib.sbx_get_particles(self._h, _ptr(x), _ptr(v), _ptr(lost)))
        return x, v, lost.astype(bool)

    def sbx_get_centres(self):
        c = np.empty((self.ngal, 3))
        _check(_lib.sbx_get_centres(self._h, _ptr(c)))
        return c

    def sbx_get_indices(self, galaxy, level):
        idx = np.empty((self.n, 3), np.int32); cls = np.empty(self.n, np.int8)
        _check(_lib.sbx_get_indices(self._h, galaxy, level, _ptr(idx), _ptr(cls)))
        return idx, cls

    def sbx_get_grid(self, galaxy, which, kind):
        """Grid as an (N, N, N) float64 array indexed [iz, iy, ix]."""
        n = self.hier[galaxy].lv[0].n
        out = np.empty((n, n, n))
        _check(_lib.sbx_get_grid(self._h, galaxy, which, kind, _ptr(out)))
        return out

    def sbx_diagnostics(self, dt):
        d = sbx_diag()
        _check(_lib.sbx_diagnostics(self._h, float(dt), C.byref(d)))
        return d.as_dict()

    def sbx_diag_log(self, max_entries=4096):
        arr = (sbx_diag * max_entries)()
        cnt = C.c_int32()
        _check(_lib.sbx_diag_log(self._h, max_entries, arr, C.byref(cnt)))
        return [arr[i].as_dict() for i in range(min(cnt.value, max_entries))]

    def sbx_profile_begin(self, max_marks=100000):
        _check(_lib.sbx_profile_begin(self._h, int(max_marks)))

    def sbx_profile_end(self):
        """{phase name: (total ms, launches)}."""
        ms = np.zeros(N_PHASES); cnt = np.zeros(N_PHASES, np.int64)
        _check(_lib.sbx_profile_end(self._h, N_PHASES, _ptr(ms), _ptr(cnt)))
        return {PHASES[i]: (float(ms[i]), int(cnt[i])) for i in range(1, N_PHASES)}

    def sbx_count_live(self):
        k = C.c_int64()
        _check(_lib.sbx_count_live(self._h, C.byref(k)))
        return k.value


class Batch:
    """A batch of contexts stepped together (sbx_batch_*)."""

    def __init__(self, contexts, stream=None):
        arr = (C.c_void_p * len(contexts))(*[c._h.value for c in contexts])
        h = C.c_void_p()
        _check(_lib.sbx_batch_create(arr, len(contexts), stream, C.byref(h)))
        self._h = h
        self.contexts = list(contexts)

    def close(self):
        if self._h:
            _lib.sbx_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sbx_batch_step(self, dt=None, nsteps=1):
        if dt is None:
            p = None
        else:
            dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, np.float64), (len(self.contexts),)))
            p = _ptr(dt)
        _check(_lib.sbx_batch_step(self._h, p, int(nsteps)))

    def sbx_batch_sync(self):
        _check(_lib.sbx_batch_sync(self._h))

    def sbx_batch_set_sort_interval(self, every):
        _check(_lib.sbx_batch_set_sort_interval(self._h, int(every)))


class Poisson:
    """Standalone isolated solves on one geometry (sbx_poisson_*)."""

    def __init__(self, n, R, q=1.0, G=1.0, h0_mode=0, prec=SBX_FP32, device=0, stream=None):
        h = C.c_void_p()
        _check(_lib.sbx_poisson_create(n, R, q, G, h0_mode, prec, device, stream, C.byref(h)))
        self._h = h
        self.n = n
        self.prec = prec

    def close(self):
        if self._h:
            _lib.sbx_poisson_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sbx_poisson_solve(self, batch, rho_ptr, phi_ptr):
        """rho_ptr, phi_ptr: device addresses (int) of batch * n^3 elements."""
        _check(_lib.sbx_poisson_solve(self._h, int(batch), C.c_void_p(rho_ptr), C.c_void_p(phi_ptr)))

    def sbx_poisson_solve_noalloc(self, batch, rho_ptr, phi_ptr):
        """As sbx_poisson_solve, with the fixed per-GPU work space (no device
        allocation; overlapping calls on one GPU race)."""
        _check(_lib.sbx_poisson_solve_noalloc(self._h, int(batch), C.c_void_p(rho_ptr),
                                              C.c_void_p(phi_ptr)))

    def sbx_poisson_green(self):
        n1 = self.n + 1
        out = np.empty((n1, n1, n1))
        rel = C.c_double()
        _check(_lib.sbx_poisson_green(self._h, _ptr(out), C.byref(rel)))
        return out, rel.value

    def sbx_poisson_bytes(self):
        return int(_lib.sbx_poisson_bytes(self._h))
