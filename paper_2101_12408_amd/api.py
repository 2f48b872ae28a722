"""Python binding of the C ABI (include/mpm.h): argument marshalling around torch tensors.

Every computation runs in libmpm.so; this module only converts parameters, hands device
pointers of torch tensors to the library, and exposes workspace fields as tensor views.
The functions keep the C names (mpm_p2g, mpm_energy_grad, mpm_hessvec, mpm_heat_apply,
mpm_g2p, mpm_step); Scene bundles a context with its workspace.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


class MpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{L.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(rc, lib, ctx=None):
    if rc != L.MPM_OK:
        msg = lib.mpm_last_error(ctx).decode()
        raise MpmError(rc, msg)


def make_params(d, precision="fp64"):
    """mpm_params from a parameter dict (keys as in mpm_scenes.DEFAULT_PARAMS)."""
    lib = L.load()
    p = L.MpmParams()
    _check(lib.mpm_params_default(C.byref(p), int(d["dim"]), int(d["n"])), lib)
    p.precision = L.MPM_FP64 if precision == "fp64" else L.MPM_MIXED
    ints = ("hess_mode", "term_mask", "momentum_fix", "wall_layers", "slab", "slab_axis", "heat",
            "gamma_by_label", "newton_max", "cg_max", "ls_max", "heat_max", "krylov")
    for k in ints:
        if k in d:
            setattr(p, k, int(d[k]))
    for k in ("dx", "dt", "bulk", "mu0", "mu_k", "mu_T0", "g0", "g1", "gT0", "gmin", "gmax", "cp", "K", "h",
              "T_amb", "b", "H", "newton_tol", "cg_rel", "ls_c1", "heat_tol", "cfl", "dt_min", "dt_max",
              "T_melt", "muh0", "lamh0", "kh", "Th0"):
        if k in d:
            setattr(p, k, float(d[k]))
    for k, ln in (("gravity", 3), ("gamma_label", 4), ("slab_lo", 3), ("slab_hi", 3)):
        if k in d:
            vals = list(d[k]) + [0.0] * ln
            getattr(p, k)[:] = [float(v) for v in vals[:ln]]
    planes = d.get("planes") or ()
    if len(planes) > 4:
        raise MpmError(L.MPM_EINVAL, "at most 4 collision planes")
    p.n_planes = len(planes)
    for k, (o, nrm, mu) in enumerate(planes):
        p.plane_o[k][:] = [float(v) for v in (list(o) + [0.0] * 3)[:3]]
        p.plane_n[k][:] = [float(v) for v in (list(nrm) + [0.0] * 3)[:3]]
        p.plane_mu[k] = float(mu)
    return p


def tiled_index(dim, n):
    """Tiled node number of every node in natural order (x fastest), as in mpm_node_index."""
    E = 4 if dim == 3 else 8
    nt = n // E
    g = np.arange(n)
    if dim == 3:
        k, j, i = np.meshgrid(g, g, g, indexing="ij")
        tile = i // E + nt * (j // E + nt * (k // E))
        loc = i % E + E * (j % E + E * (k % E))
    else:
        j, i = np.meshgrid(g, g, indexing="ij")
        tile = i // E + nt * (j // E)
        loc = i % E + E * (j % E)
    return (tile * 64 + loc).ravel()


def sample_surface(x, params, step=0):
    """Host sampler (mpm_sample_surface) around positions x (N, d) float64."""
    lib = L.load()
    x = np.ascontiguousarray(np.asarray(x, np.float64).T)
    dim, n = int(params["dim"]), int(params["n"])
    N = x.shape[1]
    lo = np.ascontiguousarray(np.asarray(list(params.get("label_lo", (0, 0, 0)))[:3] + [0] * 3, np.float64)[:3])
    hi = np.ascontiguousarray(np.asarray(list(params.get("label_hi", (0, 0, 0)))[:3] + [0] * 3, np.float64)[:3])
    cnt = C.c_int64(0)
    radius = float(params.get("ls_radius") or 0.0)
    density = float(params.get("sample_density") or 0.0)
    seed = int(params.get("seed", 0))
    cap = max(16, 2 * N + 4096)    # grown to the exact count if the first call overflows
    for _ in range(3):
        s = np.zeros((dim, cap))
        dA = np.zeros((dim, cap))
        lab = np.zeros(cap, np.int32)
        _check(lib.mpm_sample_surface(dim, n, x.ctypes.data, N, radius, density, seed, int(step),
                                      lo.ctypes.data, hi.ctypes.data, s.ctypes.data, dA.ctypes.data,
                                      lab.ctypes.data, cap, C.byref(cnt)), lib)
        if cnt.value <= cap:
            S = cnt.value
            return dict(s=np.ascontiguousarray(s[:, :S].T), dA=np.ascontiguousarray(dA[:, :S].T),
                        label=lab[:S].copy())
        cap = cnt.value
    raise MpmError(L.MPM_ENOMEM, "sample buffer")


class Scene:
    """One simulation context: parameters, a device workspace and the C context."""

    def __init__(self, params, cap_part, cap_surf, precision="fp64", device="cuda"):
        import torch
        self.torch = torch
        self.lib = L.load()
        self.params = dict(params)
        self.p = make_params(params, precision)
        self.dim, self.n = int(self.p.dim), int(self.p.n)
        self.nn = self.n ** self.dim
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.precision = precision
        nbytes = C.c_size_t(0)
        _check(self.lib.mpm_workspace_bytes(C.byref(self.p), int(cap_part), int(cap_surf), C.byref(nbytes)), self.lib)
        self.ws_bytes = nbytes.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        self.ws_off = (-base) % 256
        self.ws_base = base + self.ws_off
        ctx = C.c_void_p()
        _check(self.lib.mpm_ctx_create(C.byref(self.p), C.c_void_p(self.ws_base), self.ws_bytes, int(cap_part),
                                       int(cap_surf), C.byref(ctx)), self.lib)
        self.ctx = ctx
        self.cap_part, self.cap_surf = int(cap_part), int(cap_surf)
        self._keep = []

    def close(self):
        if self.ctx:
            self.lib.mpm_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, **kw):
        self.params.update(kw)
        prec = self.precision
        self.p = make_params(self.params, prec)
        _check(self.lib.mpm_ctx_set_params(self.ctx, C.byref(self.p)), self.lib, self.ctx)

    # ---- marshalling ------------------------------------------------------------------
    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def particles_struct(self, P):
        st = L.MpmParticles()
        st.n = int(P["m"].shape[0])
        for k in ("x", "v", "A", "J", "V0", "m", "T", "gradT", "F"):
            if k == "F" and k not in P:
                continue
            t = P[k]
            assert t.dtype == self.dtype and t.is_contiguous() and t.is_cuda, k
            setattr(st, k, t.data_ptr())
        return st

    def surface_struct(self, S):
        st = L.MpmSurface()
        if S is None:
            st.n = 0
            return st
        st.n = int(S["s"].shape[1])
        st.s = S["s"].data_ptr() if st.n else None
        st.dA = S["dA"].data_ptr() if st.n else None
        st.label = S["label"].data_ptr() if (st.n and S.get("label") is not None) else None
        return st

    def to_device(self, P=None, S=None):
        """Converts natural-order numpy particle / surface dicts to SoA device tensors."""
        torch = self.torch
        out = []
        if P is not None:
            N = P["x"].shape[0]
            d = self.dim
            f = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=self.dtype).contiguous()
            Pd = dict(x=f(P["x"].T), v=f(P["v"].T), A=f(P["A"].reshape(N, d * d).T), J=f(P["J"]),
                      V0=f(P["V0"]), m=f(P["m"]), T=f(P["T"]), gradT=f(P["gradT"].T))
            if "F" in P:
                Pd["F"] = f(P["F"].reshape(N, d * d).T)
            out.append(Pd)
        if S is not None:
            f = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=self.dtype).contiguous()
            lab = S.get("label")
            lab = np.zeros(S["s"].shape[0], np.int32) if lab is None else lab
            out.append(dict(s=f(S["s"].T), dA=f(S["dA"].T),
                            label=torch.from_numpy(np.ascontiguousarray(lab.astype(np.int32))).cuda()))
        return out[0] if len(out) == 1 else tuple(out)

    def autotune(self):
        """mpm_autotune after p2g: {class: (chosen run length, {run: microseconds})}."""
        t = L.MpmTuning()
        _check(self.lib.mpm_autotune(self.ctx, self.stream(), C.byref(t)), self.lib, self.ctx)
        out = {}
        for k, name in enumerate(("energy", "hess", "heat")):
            if t.run[k]:
                out[name] = (int(t.run[k]), {int(t.cand[j]): round(float(t.us[k][j]), 2) for j in range(t.ncand)})
        return out

    def tuning_set(self, run=None):
        arr = None if run is None else (C.c_int32 * 3)(*run)
        _check(self.lib.mpm_tuning_set(self.ctx, arr), self.lib, self.ctx)

    def sample_surface(self, P, step=0, cap=None):
        """Device sampler (mpm_sample_surface_dev) around the device positions P["x"]
        ([dim][N] of the scene's dtype): the host sampler's samples, as device tensors
        {s (dim, S), dA (dim, S), label (S,)} ready for step / p2g."""
        torch = self.torch
        prm = self.params
        st = L.MpmParticles()
        st.n = int(P["x"].shape[1])
        assert P["x"].dtype == self.dtype and P["x"].is_contiguous() and P["x"].is_cuda
        st.x = P["x"].data_ptr()
        lo = (C.c_double * 3)(*(list(prm.get("label_lo", (0, 0, 0)))[:3] + [0.0] * 3)[:3])
        hi = (C.c_double * 3)(*(list(prm.get("label_hi", (0, 0, 0)))[:3] + [0.0] * 3)[:3])
        radius = float(prm.get("ls_radius") or 0.0)
        density = float(prm.get("sample_density") or 0.0)
        seed = int(prm.get("seed", 0))
        cap = self.cap_surf if cap is None else int(cap)
        cnt = C.c_int64(0)
        for _ in range(2):
            s = torch.empty(self.dim * max(cap, 1), dtype=self.dtype, device="cuda")
            dA = torch.empty_like(s)
            lab = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
            _check(self.lib.mpm_sample_surface_dev(self.ctx, C.byref(st), radius, density, seed, int(step), lo, hi,
                                                   s.data_ptr(), dA.data_ptr(), lab.data_ptr(), cap, C.byref(cnt),
                                                   self.stream()), self.lib, self.ctx)
            S = cnt.value
            if S <= cap:
                d = self.dim
                return dict(s=s[:d * S].view(d, S), dA=dA[:d * S].view(d, S), label=lab[:S])
            cap = S
        raise MpmError(L.MPM_ENOMEM, "sample buffer")

    def grid_vector(self, ncomp=None):
        ncomp = self.dim if ncomp is None else ncomp
        return self.torch.zeros((ncomp, self.nn), dtype=self.dtype, device="cuda")

    # ---- the ABI calls ------------------------------------------------------------------
    def p2g(self, P, S=None):
        self._P = self.particles_struct(P)
        self._S = self.surface_struct(S)
        self._keep = [P, S]
        _check(self.lib.mpm_p2g(self.ctx, C.byref(self._P), C.byref(self._S), self.stream()), self.lib, self.ctx)

    def energy_grad(self, v, grad, energy=None):
        torch = self.torch
        e = torch.zeros(1, dtype=torch.float64, device="cuda") if energy is None else energy
        _check(self.lib.mpm_energy_grad(self.ctx, v.data_ptr(), e.data_ptr(), grad.data_ptr(), self.stream()),
               self.lib, self.ctx)
        return e

    def hessvec(self, vlin, w, alpha, out):
        _check(self.lib.mpm_hessvec(self.ctx, vlin.data_ptr(), w.data_ptr(), float(alpha), out.data_ptr(),
                                    self.stream()), self.lib, self.ctx)

    def heat_apply(self, T, out):
        _check(self.lib.mpm_heat_apply(self.ctx, T.data_ptr(), out.data_ptr(), self.stream()), self.lib, self.ctx)

    def g2p(self, vhat, That, P):
        st = self.particles_struct(P)
        _check(self.lib.mpm_g2p(self.ctx, vhat.data_ptr(), That.data_ptr() if That is not None else None,
                                C.byref(st), self.stream()), self.lib, self.ctx)

    def solve_momentum(self, check=True):
        rc = self.lib.mpm_solve_momentum(self.ctx, self.stream())
        if check:
            _check(rc, self.lib, self.ctx)
        return rc

    def solve_heat(self, check=True):
        rc = self.lib.mpm_solve_heat(self.ctx, self.stream())
        if check:
            _check(rc, self.lib, self.ctx)
        return rc

    def step(self, P, S=None, implicit=True, check=True):
        return mpm_step([self], [P], [S], implicit=implicit, check=check)

    def status(self):
        return self.lib.mpm_scene_status(self.ctx, self.stream())

    def stats(self):
        st = L.MpmStats()
        _check(self.lib.mpm_get_stats(self.ctx, C.byref(st)), self.lib, self.ctx)
        out = {k: getattr(st, k) for k, _ in L.MpmStats._fields_}
        out["momentum"] = list(st.momentum)
        return out

    def timing(self, enable=True):
        """Starts (and resets) or stops per-kernel-class HIP-event timing."""
        _check(self.lib.mpm_timing(self.ctx, 1 if enable else 0), self.lib, self.ctx)

    def timing_read(self, work=False):
        """{kernel class: (total ms, launches)} since timing was enabled; with work=True
        (total ms, launches) over the launches that did work (a called-off CG's launches,
        which return at once, left out)."""
        n = len(L.KERNEL_CLASSES)
        ms, cnt = (C.c_double * n)(), (C.c_int64 * n)()
        wms, wcnt = (C.c_double * n)(), (C.c_int64 * n)()
        _check(self.lib.mpm_timing_read(self.ctx, C.cast(ms, C.c_void_p), C.cast(cnt, C.c_void_p),
                                        C.cast(wms, C.c_void_p), C.cast(wcnt, C.c_void_p)), self.lib, self.ctx)
        if work:
            return {k: (wms[i], wcnt[i]) for i, k in enumerate(L.KERNEL_CLASSES)}
        return {k: (ms[i], cnt[i]) for i, k in enumerate(L.KERNEL_CLASSES)}

    def view(self, field, count=None):
        """Workspace field as a tensor view (no copy)."""
        torch = self.torch
        ptr = C.c_void_p()
        _check(self.lib.mpm_grid_view(self.ctx, int(field), C.byref(ptr)), self.lib, self.ctx)
        off = ptr.value - self.ws.data_ptr()
        d, nn = self.dim, self.nn
        st = self.stats()
        if field in (L.F_MOM, L.F_VN, L.F_VHAT, L.F_MOM_DIAG):
            dt, shape = self.dtype, (d, nn)
        elif field == L.F_FREE:
            dt, shape = torch.uint8, (nn,)
        elif field == L.F_PARENT:
            dt, shape = torch.int32, (st["n_surf"],)
        elif field in (L.F_COUNT, L.F_PERM):
            dt, shape = torch.int32, (st["n_part"],)
        elif field == L.F_KSURF:
            dt, shape = self.dtype, (st["n_surf"],)
        else:
            dt, shape = self.dtype, (nn,)
        esz = torch.tensor([], dtype=dt).element_size()
        nbytes = int(np.prod(shape)) * esz
        return self.ws[off:off + nbytes].view(dt).view(shape)


def mpm_step(scenes, Ps, Ss, implicit=True, check=True):
    """mpm_step over a batch of scenes (each with its own context)."""
    lib = L.load()
    n = len(scenes)
    ctxs = (C.c_void_p * n)(*[s.ctx.value for s in scenes])
    pstructs = [s.particles_struct(P) for s, P in zip(scenes, Ps)]
    sstructs = [s.surface_struct(S) for s, S in zip(scenes, Ss)]
    parr = (C.POINTER(L.MpmParticles) * n)(*[C.pointer(p) for p in pstructs])
    sarr = (C.POINTER(L.MpmSurface) * n)(*[C.pointer(p) for p in sstructs])
    rc = lib.mpm_step(ctxs, parr, sarr, n, 1 if implicit else 0, scenes[0].stream())
    if check and rc != L.MPM_OK:
        bad = next((s for s in scenes if s.stats()["status"] != L.MPM_OK), scenes[0])
        _check(rc, lib, bad.ctx)
    return rc


def step_noalloc(params, P, S=None, implicit=True, precision="fp64", check=True):
    """mpm_step_noalloc: one step of one scene on the library's static scratch (no context,
    no workspace).  P, S: device tensor dicts as from Scene.to_device.  Returns (status,
    scratch bytes)."""
    import torch
    lib = L.load()
    p = make_params(params, precision)
    dtype = torch.float64 if precision == "fp64" else torch.float32
    pst = L.MpmParticles()
    pst.n = int(P["m"].shape[0])
    for k in ("x", "v", "A", "J", "V0", "m", "T", "gradT"):
        t = P[k]
        assert t.dtype == dtype and t.is_contiguous() and t.is_cuda, k
        setattr(pst, k, t.data_ptr())
    sst = L.MpmSurface()
    if S is not None and int(S["s"].shape[1]):
        sst.n = int(S["s"].shape[1])
        sst.s, sst.dA = S["s"].data_ptr(), S["dA"].data_ptr()
        sst.label = S["label"].data_ptr() if S.get("label") is not None else None
    nb = C.c_size_t(0)
    rc = lib.mpm_step_noalloc(C.byref(p), C.byref(pst), C.byref(sst), 1 if implicit else 0,
                              C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(nb))
    if check:
        _check(rc, lib)
    return rc, nb.value


def batch_config(max_concurrent):
    """Maximum number of scenes mpm_step advances at once (process-wide)."""
    lib = L.load()
    _check(lib.mpm_batch_config(int(max_concurrent)), lib)


# C-named functional aliases
def mpm_p2g(scene, P, S=None):
    return scene.p2g(P, S)


def mpm_energy_grad(scene, v, grad, energy=None):
    return scene.energy_grad(v, grad, energy)


def mpm_hessvec(scene, vlin, w, alpha, out):
    return scene.hessvec(vlin, w, alpha, out)


def mpm_heat_apply(scene, T, out):
    return scene.heat_apply(T, out)


def mpm_g2p(scene, vhat, That, P):
    return scene.g2p(vhat, That, P)


class Server:
    """Serving runtime (mpm_server_*): continuous batching of step requests over a device
    arena of budget_bytes; max_concurrent requests run at once on their own streams."""

    def __init__(self, budget_bytes, max_concurrent=8, device="cuda"):
        import torch
        self.lib = L.load()
        self.arena = torch.empty(int(budget_bytes) + 256, dtype=torch.uint8, device=device)
        base = self.arena.data_ptr()
        base += (-base) % 256
        srv = C.c_void_p()
        _check(self.lib.mpm_server_create(C.c_void_p(base), int(budget_bytes), int(max_concurrent), C.byref(srv)),
               self.lib)
        self.srv = srv

    @staticmethod
    def clock():
        return L.load().mpm_server_clock()

    @staticmethod
    def soa(P, dim):
        """Host particle dict (x (N,d), v, A (N,d,d), J, V0, m, T, gradT) as the contiguous
        SoA double arrays a request reads."""
        N, d = len(P["m"]), dim
        soa = dict(x=np.asarray(P["x"], np.float64).reshape(N, d).T, v=np.asarray(P["v"], np.float64).reshape(N, d).T,
                   A=np.asarray(P["A"], np.float64).reshape(N, d * d).T, J=np.asarray(P["J"], np.float64),
                   V0=np.asarray(P["V0"], np.float64), m=np.asarray(P["m"], np.float64),
                   T=np.asarray(P["T"], np.float64), gradT=np.asarray(P["gradT"], np.float64).reshape(N, d).T)
        return {k: np.ascontiguousarray(v) for k, v in soa.items()}

    def submit(self, rid, params, P=None, n_steps=1, precision="mixed", implicit=True, keep_result=False,
               first_step=0, soa=None, borrow=False):
        """Queues one request.  P: host particle dict, or soa: arrays from Server.soa().
        borrow: the server reads soa in place; the caller keeps the arrays alive and
        unchanged until the request completes."""
        p = make_params(params, precision)
        d = int(p.dim)
        if soa is None:
            soa = self.soa(P, d)
            borrow = False
        N = len(soa["m"])
        r = L.MpmRequest()
        r.id, r.params, r.n_steps, r.implicit, r.keep_result = int(rid), p, int(n_steps), int(bool(implicit)), \
            int(bool(keep_result))
        r.borrow = int(bool(borrow))
        r.n_part, r.seed, r.first_step = N, int(params.get("seed", 0)), int(first_step)
        r.ls_radius = float(params.get("ls_radius") or 0.0)
        r.sample_density = float(params.get("sample_density") or 0.0)
        lo = list(params.get("label_lo", (0, 0, 0)))[:3] + [0.0] * 3
        hi = list(params.get("label_hi", (0, 0, 0)))[:3] + [0.0] * 3
        r.label_lo = (C.c_double * 3)(*lo[:3])
        r.label_hi = (C.c_double * 3)(*hi[:3])
        for k, v in soa.items():
            setattr(r, k, v.ctypes.data)
        _check(self.lib.mpm_server_submit(self.srv, C.byref(r)), self.lib)   # copies the arrays

    def poll(self, cap=4096):
        out = (L.MpmCompletion * cap)()
        n = C.c_int32(0)
        _check(self.lib.mpm_server_poll(self.srv, out, cap, C.byref(n)), self.lib)
        return [{f: getattr(out[k], f) for f, _ in L.MpmCompletion._fields_} for k in range(n.value)]

    def wait(self, timeout=-1.0):
        return self.lib.mpm_server_wait(self.srv, float(timeout))

    def result(self, rid, N, dim):
        x, v = np.zeros((dim, N)), np.zeros((dim, N))
        A, gT = np.zeros((dim * dim, N)), np.zeros((dim, N))
        J, T = np.zeros(N), np.zeros(N)
        rc = self.lib.mpm_server_result(self.srv, int(rid), x.ctypes.data, v.ctypes.data, A.ctypes.data,
                                        J.ctypes.data, T.ctypes.data, gT.ctypes.data)
        return rc, dict(x=x.T.copy(), v=v.T.copy(), A=A.T.reshape(N, dim, dim).copy(), J=J, T=T, gradT=gT.T.copy())

    def info(self):
        i = L.MpmServerInfo()
        _check(self.lib.mpm_server_info_get(self.srv, C.byref(i)), self.lib)
        return {f: getattr(i, f) for f, _ in L.MpmServerInfo._fields_ if f != "pad_"}

    def close(self):
        if self.srv:
            self.lib.mpm_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
