"""Python face of libfockmi: plans over torch device tensors.

PyTorch supplies device memory and the current stream; every computation runs
in the HIP library. Tensors are complex128, contiguous, on the plan's device,
shaped [nk][nbands][n1][n2][n3].
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as N

PRECISIONS = {"fp64": N.FOCK_FP64, "fp32": N.FOCK_FP32_COMP, "fp64f": N.FOCK_FP64_FUSED}


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A set of cells (grid, lattice, k-points, bands, screening) prepared on one GPU.

    cells : list of dicts with keys n (int or 3-tuple), a (3x3 rows), kpts ([nk][3]),
            nb, omega, gs (default 2.0), and optionally src: the k indices of a
            down-sampled source sub-mesh (the pair sum runs over them with weight 1/len(src))
    prec  : "fp64" (plain staged FP64 path), "fp32" (fused complex64 pair FFTs with
            compensated FP64 accumulation) or "fp64f" (fused kernel in FP64 throughout for
            cubic grids of length 16, 20, 24; other cells take the plain path)
    """

    def __init__(self, cells, prec="fp64", tune_cache=None):
        self._lib = N.lib()
        if isinstance(cells, dict):
            cells = [cells]
        self.prec = prec
        self.cells = []
        descs = (N.CellDesc * len(cells))()
        self._keep = []
        for ci, c in enumerate(cells):
            n = c["n"]
            n = (int(n),) * 3 if np.isscalar(n) else tuple(int(x) for x in n)
            a = np.ascontiguousarray(np.asarray(c["a"], dtype=np.float64).reshape(3, 3))
            kpts = np.ascontiguousarray(np.asarray(c["kpts"], dtype=np.float64).reshape(-1, 3))
            self._keep.append(kpts)
            d = descs[ci]
            for i in range(3):
                d.n[i] = n[i]
                for j in range(3):
                    d.a[i][j] = float(a[i, j])
            d.nk = len(kpts)
            d.kpts = kpts.ctypes.data_as(C.POINTER(C.c_double))
            d.nb = int(c["nb"])
            d.omega = float(c["omega"])
            d.gs = float(c.get("gs", 2.0))
            src = c.get("src")
            if src is not None:
                src = np.ascontiguousarray(np.asarray(src, dtype=np.int32).reshape(-1))
                self._keep.append(src)
                d.nsrc = len(src)
                d.src = src.ctypes.data_as(C.POINTER(C.c_int))
            self.cells.append(dict(n=n, a=a, kpts=kpts, nk=len(kpts), nb=int(c["nb"]), omega=float(c["omega"]),
                                   gs=float(c.get("gs", 2.0)), nr=n[0] * n[1] * n[2],
                                   vol=abs(float(np.linalg.det(a))),
                                   src=None if src is None else [int(x) for x in src]))
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = C.c_void_p()
        path = tune_cache.encode() if tune_cache else None
        N.check(self._lib.fock_plan_create(descs, len(cells), PRECISIONS[prec], path, C.byref(h)))
        self._h = h

    # ------------------------------------------------------------------ utils
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fock_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, t, cell, nb=None, name="tensor"):
        c = self.cells[cell]
        if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
            raise TypeError(f"{name} must be a complex128 CUDA tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, plan on {self.device}")
        exp = (c["nk"],) + ((nb,) if nb is not None else (t.shape[1],)) + c["n"]
        if tuple(t.shape) != exp:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {exp}")
        return t

    def profile(self, enable=True):
        """Bracket the dominant kernel's launches with HIP events on the caller's stream."""
        N.check(self._lib.fock_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self, reset=True):
        """(summed kernel milliseconds, number of bracketed launches)."""
        ms = C.c_double()
        n = C.c_longlong()
        N.check(self._lib.fock_profile_read(self._h, C.byref(ms), C.byref(n), 1 if reset else 0))
        return ms.value, n.value

    def profile_fallbacks(self, reset=True):
        """Split 32^3 launches (counted while profiling) whose result came from the lockstep form."""
        n = C.c_longlong()
        N.check(self._lib.fock_profile_fallbacks(self._h, C.byref(n), 1 if reset else 0))
        return n.value

    # ------------------------------------------------------------- operations
    def apply(self, u, phi=None, cell=0, out=None):
        """V_x[u] phi (phi defaults to u)."""
        c = self.cells[cell]
        self._check(u, cell, c["nb"], "u")
        phi = u if phi is None else self._check(phi, cell, None, "phi")
        if out is None:
            out = torch.empty_like(phi)
        else:
            self._check(out, cell, phi.shape[1], "out")
        N.check(self._lib.fock_apply(self._h, cell, _ptr(u), _ptr(phi), phi.shape[1], _ptr(out), _stream()))
        return out

    def apply_krange(self, u, k0, nk_out, phi=None, cell=0, out=None):
        """V_x[u] phi for the output k-points k0 .. k0 + nk_out - 1 (phi: those k-points;
        default u[k0:k0 + nk_out]); one GPU's share of a k-point decomposition."""
        c = self.cells[cell]
        self._check(u, cell, c["nb"], "u")
        phi = u[k0:k0 + nk_out] if phi is None else phi
        if not isinstance(phi, torch.Tensor) or phi.dtype != torch.complex128 or not phi.is_cuda \
                or not phi.is_contiguous() or tuple(phi.shape[2:]) != c["n"] or phi.shape[0] != nk_out:
            raise ValueError("phi must be a contiguous complex128 CUDA tensor [nk_out][nphi][n1][n2][n3]")
        out = torch.empty_like(phi) if out is None else out
        N.check(self._lib.fock_apply_krange(self._h, cell, _ptr(u), int(k0), int(nk_out), _ptr(phi), phi.shape[1],
                                            _ptr(out), _stream()))
        return out

    def energy(self, u, cell=0):
        """E_x of u as a complex number (imaginary part is a reality check)."""
        c = self.cells[cell]
        self._check(u, cell, c["nb"], "u")
        re, im = C.c_double(), C.c_double()
        N.check(self._lib.fock_energy(self._h, cell, _ptr(u), C.byref(re), C.byref(im), _stream()))
        return complex(re.value, im.value)

    def energy_vjp(self, u, g_e=1.0, cell=0, out=None):
        """g_e dE_x/du (torch convention) for the cotangent g_e of E_x."""
        c = self.cells[cell]
        self._check(u, cell, c["nb"], "u")
        out = torch.empty_like(u) if out is None else self._check(out, cell, c["nb"], "out")
        N.check(self._lib.fock_energy_vjp(self._h, cell, _ptr(u), float(g_e), _ptr(out), _stream()))
        return out

    def vjp(self, u, phi, g, cell=0, need_u=True, need_phi=True):
        """(g_u, g_phi) of y = V_x[u] phi for the cotangent g of y (torch convention)."""
        c = self.cells[cell]
        self._check(u, cell, c["nb"], "u")
        self._check(phi, cell, None, "phi")
        self._check(g, cell, phi.shape[1], "g")
        gu = torch.empty_like(u) if need_u else None
        gp = torch.empty_like(phi) if need_phi else None
        N.check(self._lib.fock_vjp(self._h, cell, _ptr(u), _ptr(phi), phi.shape[1], _ptr(g), _ptr(gu), _ptr(gp),
                                   _stream()))
        return gu, gp

    def taylor_step(self, psi, a_over_c, dt, alpha, vloc=None, order=4, cell=0, want_norm=True):
        """psi <- T_order(-i dt h) psi in place; returns max |norm - 1| (or None)."""
        c = self.cells[cell]
        self._check(psi, cell, c["nb"], "psi")
        av = (C.c_double * 3)(*[float(x) for x in a_over_c])
        dev = C.c_double()
        if vloc is not None:
            if vloc.dtype != torch.float64 or not vloc.is_cuda or vloc.numel() != c["nr"]:
                raise ValueError("vloc must be a float64 CUDA tensor with N_r entries")
        st = self._lib.taylor_step(self._h, cell, _ptr(psi), _ptr(vloc) if vloc is not None else None, av,
                                   float(dt), float(alpha), int(order), C.byref(dev) if want_norm else None,
                                   _stream())
        N.check(st)
        return dev.value if want_norm else None

    def taylor_step_pc(self, psi, a_now, a_mid, dt, alpha, vloc=None, order=4, cell=0, want_norm=True):
        """Predictor-corrector step in place: predictor with A(t_n) and V_x[psi(t_n)], corrector with
        A(t_n + dt/2) and the average of V_x[psi(t_n)] and V_x[psi_pred]; returns max |norm - 1| (or None)."""
        c = self.cells[cell]
        self._check(psi, cell, c["nb"], "psi")
        an = (C.c_double * 3)(*[float(x) for x in a_now])
        am = (C.c_double * 3)(*[float(x) for x in a_mid])
        dev = C.c_double()
        if vloc is not None:
            if vloc.dtype != torch.float64 or not vloc.is_cuda or vloc.numel() != c["nr"]:
                raise ValueError("vloc must be a float64 CUDA tensor with N_r entries")
        N.check(self._lib.taylor_step_pc(self._h, cell, _ptr(psi), _ptr(vloc) if vloc is not None else None, an, am,
                                         float(dt), float(alpha), int(order), C.byref(dev) if want_norm else None,
                                         _stream()))
        return dev.value if want_norm else None

    def taylor_step_vjp(self, psi_n, a_over_c, dt, alpha, g_next, vloc=None, order=4, cell=0):
        """(g_psi_n, g_a) for one Taylor step."""
        c = self.cells[cell]
        self._check(psi_n, cell, c["nb"], "psi_n")
        self._check(g_next, cell, c["nb"], "g_next")
        av = (C.c_double * 3)(*[float(x) for x in a_over_c])
        ga = (C.c_double * 3)()
        gpsi = torch.empty_like(psi_n)
        N.check(self._lib.taylor_step_vjp(self._h, cell, _ptr(psi_n), _ptr(vloc) if vloc is not None else None, av,
                                          float(dt), float(alpha), int(order), _ptr(g_next), _ptr(gpsi), ga,
                                          _stream()))
        return gpsi, np.array([ga[0], ga[1], ga[2]])

    def energy_functional(self, psi, a_over_c, alpha, vloc=None, cell=0, want_grad=False):
        """E[psi; a] = (g_s/N_k)(Omega/N_r) sum conj(psi)(T[a] + v_loc) psi + alpha E_x[psi].

        With want_grad, returns (E, dE/dpsi, dE/da)."""
        c = self.cells[cell]
        self._check(psi, cell, c["nb"], "psi")
        av = (C.c_double * 3)(*[float(x) for x in a_over_c])
        e = C.c_double()
        g = torch.empty_like(psi) if want_grad else None
        ga = (C.c_double * 3)()
        N.check(self._lib.taylor_energy(self._h, cell, _ptr(psi), _ptr(vloc) if vloc is not None else None, av,
                                        float(alpha), C.byref(e), _ptr(g), ga if want_grad else None, _stream()))
        return (e.value, g, np.array([ga[0], ga[1], ga[2]])) if want_grad else e.value

    def excitation_energy(self, psi_t, a_t, psi_0, a_0, alpha, vloc=None, cell=0):
        """E[psi_t; a_t] - E[psi_0; a_0], both reduced and subtracted in double-double."""
        c = self.cells[cell]
        self._check(psi_t, cell, c["nb"], "psi_t")
        self._check(psi_0, cell, c["nb"], "psi_0")
        at = (C.c_double * 3)(*[float(x) for x in a_t])
        a0 = (C.c_double * 3)(*[float(x) for x in a_0])
        e = C.c_double()
        N.check(self._lib.taylor_excitation_energy(self._h, cell, _ptr(psi_t), at, _ptr(psi_0), a0,
                                                   _ptr(vloc) if vloc is not None else None, float(alpha),
                                                   C.byref(e), _stream()))
        return e.value

    def energy_functional_vjp(self, psi, a_over_c, alpha, g_e=1.0, vloc=None, cell=0):
        """(g_e dE/dpsi, g_e dE/d(A/c)) of the energy functional for its cotangent g_e."""
        c = self.cells[cell]
        self._check(psi, cell, c["nb"], "psi")
        av = (C.c_double * 3)(*[float(x) for x in a_over_c])
        g = torch.empty_like(psi)
        ga = (C.c_double * 3)()
        N.check(self._lib.taylor_energy_vjp(self._h, cell, _ptr(psi), _ptr(vloc) if vloc is not None else None, av,
                                            float(alpha), float(g_e), _ptr(g), ga, _stream()))
        return g, np.array([ga[0], ga[1], ga[2]])

    def current(self, psi, a_over_c, cell=0):
        """J(t) of Eqs. (3)-(4) (velocity gauge, no nonlocal pseudopotential, electron charge -1):
        -(1/Omega) (g_s/N_k) sum_{k,b} int_cell Re[psi* (-i grad + A/c) psi] dr = -(1/Omega) dE/d(A/c)."""
        c = self.cells[cell]
        self._check(psi, cell, c["nb"], "psi")
        av = (C.c_double * 3)(*[float(x) for x in a_over_c])
        j = (C.c_double * 3)()
        N.check(self._lib.taylor_current(self._h, cell, _ptr(psi), av, j, _stream()))
        return np.array([j[0], j[1], j[2]])

    def orthonormalize(self, psi, cell=0):
        c = self.cells[cell]
        self._check(psi, cell, c["nb"], "psi")
        N.check(self._lib.fock_orthonormalize(self._h, cell, _ptr(psi), _stream()))
        return psi

    def eigensolve(self, u, phi=None, vloc=None, a_over_c=(0.0, 0.0, 0.0), alpha=0.25, tol=1e-8, maxit=200, cell=0):
        """The nb lowest eigenpairs of h = T[A/c] + v_loc + alpha V_x[u] at every k (Eq. (25)).

        phi: starting block (default: a copy of u); returns (phi, eigenvalues [nk][nb],
        residual norms [nk][nb], iterations, converged)."""
        c = self.cells[cell]
        self._check(u, cell, c["nb"], "u")
        phi = u.clone() if phi is None else phi
        self._check(phi, cell, c["nb"], "phi")
        if vloc is not None:
            if vloc.dtype != torch.float64 or not vloc.is_cuda or vloc.numel() != c["nr"] or not vloc.is_contiguous():
                raise ValueError("vloc must be a contiguous float64 CUDA tensor with N_r entries")
        av = (C.c_double * 3)(*[float(x) for x in a_over_c])
        nkb = c["nk"] * c["nb"]
        ev = (C.c_double * nkb)()
        rs = (C.c_double * nkb)()
        it = C.c_int()
        st = N.check(self._lib.fock_eigensolve(self._h, cell, _ptr(u), _ptr(vloc) if vloc is not None else None, av,
                                               float(alpha), _ptr(phi), float(tol), int(maxit), ev, rs,
                                               C.byref(it), _stream()))
        shape = (c["nk"], c["nb"])
        return (phi, np.array(ev[:]).reshape(shape), np.array(rs[:]).reshape(shape), it.value,
                st == N.FOCK_OK)

    def excited_density(self, phi, psi, cell=0):
        """n_ex of Eq. (26) (bohr^-3) for eigenvectors phi and orbitals psi."""
        c = self.cells[cell]
        self._check(phi, cell, c["nb"], "phi")
        self._check(psi, cell, c["nb"], "psi")
        out = C.c_double()
        N.check(self._lib.fock_excited_density(self._h, cell, _ptr(phi), _ptr(psi), C.byref(out), _stream()))
        return out.value

    def apply_batched(self, us, phis=None):
        """All cells in one persistent launch: returns [V_x[u_c] phi_c for each cell c]."""
        nc = len(self.cells)
        phis = us if phis is None else phis
        outs = []
        up = (C.c_void_p * nc)()
        pp = (C.c_void_p * nc)()
        op = (C.c_void_p * nc)()
        npv = (C.c_int * nc)()
        for ci in range(nc):
            self._check(us[ci], ci, self.cells[ci]["nb"], "u")
            self._check(phis[ci], ci, None, "phi")
            o = torch.empty_like(phis[ci])
            outs.append(o)
            up[ci] = us[ci].data_ptr()
            pp[ci] = phis[ci].data_ptr()
            op[ci] = o.data_ptr()
            npv[ci] = phis[ci].shape[1]
        N.check(self._lib.fock_apply_batched(self._h, up, pp, npv, op, _stream()))
        return outs
