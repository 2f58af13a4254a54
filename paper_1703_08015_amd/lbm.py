"""Python binding of liblbm (``include/lbm.h``): argument marshalling only.

Every computation runs in the HIP library; torch supplies device memory (the
solver workspace and dense fields) and the HIP stream.  The library must have
been built (``paper_1703_08015_amd.build``): a missing library raises instead
of falling back to anything else.
"""
import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lbm.h")

LBM_OK = 0
LBM_ERR_ARG = -1
LBM_ERR_SHAPE = -2
LBM_ERR_UNSUPPORTED = -3
LBM_ERR_HIP = -4
LBM_ERR_NONFINITE = -5
LBM_ERR_STATE = -6
LBM_ERR_NOMEM = -7

STORAGE = {"f64": 0, "f32": 1, "f16": 2}
ORDER = {"morton": 0, "rowmajor": 1}
KERNEL = {"auto": 0, "generic": 1, "scalar": 2, "shuffle": 3}
STORE_POLICY = {"auto": 0, "regular": 1, "nontemporal": 2}
MODEL = {"quasi-compressible": 0, "quasi": 0, "incompressible": 1}
PATTERN = {"two-copy": 0, "single-copy": 1}
COLLISION = {"bgk": 0, "mrt": 1}


class LbmError(RuntimeError):
    def __init__(self, code, where, detail):
        super().__init__("%s failed (%d): %s" % (where, code, detail))
        self.code = code


class TilesInfo(ctypes.Structure):
    _fields_ = [
        ("shape", ctypes.c_int32 * 3), ("grid", ctypes.c_int32 * 3), ("tile", ctypes.c_int32 * 3),
        ("tgrid", ctypes.c_int32 * 3), ("periodic", ctypes.c_uint32), ("words", ctypes.c_int32),
        ("n_samples", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("n_tiles", ctypes.c_int64), ("n_ftiles", ctypes.c_int64), ("n_fluid", ctypes.c_int64),
        ("n_nodes", ctypes.c_int64), ("phi", ctypes.c_double), ("phi_t", ctypes.c_double),
        ("tiles_ratio", ctypes.c_double), ("alpha_m", ctypes.c_double),
    ]


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("storage", ctypes.c_int32), ("tau", ctypes.c_double),
        ("g", ctypes.c_double * 3), ("rho0", ctypes.c_double), ("f16_scale_log2", ctypes.c_int32),
        ("tiles_per_block", ctypes.c_int32), ("tile_order", ctypes.c_int32), ("step_kernel", ctypes.c_int32),
        ("store_policy", ctypes.c_int32), ("persistent", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
        ("model", ctypes.c_int32), ("pattern", ctypes.c_int32), ("collision", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("mrt_rates", ctypes.c_double * 5),
    ]


_lib = None


def header_functions():
    """Names of the functions ``include/lbm.h`` declares."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


def lib():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbm.so is not built (%s); run paper_1703_08015_amd.build.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        PP = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "lbm_lattice": (ctypes.c_int, [I32, P, P, P]),
            "lbm_tiles_build": (ctypes.c_int, [P, P, P, U32, PP]),
            "lbm_tiles_info": (ctypes.c_int, [P, ctypes.POINTER(TilesInfo)]),
            "lbm_tiles_export": (ctypes.c_int, [P, P, P, P, P]),
            "lbm_tiles_concat": (ctypes.c_int, [P, I32, PP]),
            "lbm_tiles_free": (None, [P]),
            "lbm_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
            "lbm_create": (ctypes.c_int, [P, ctypes.POINTER(Params), P, ctypes.c_size_t, P, PP]),
            "lbm_destroy": (None, [P]),
            "lbm_set_stream": (ctypes.c_int, [P, P]),
            "lbm_set_sample_force": (ctypes.c_int, [P, P]),
            "lbm_set_lid": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, P]),
            "lbm_set_active": (ctypes.c_int, [P, P]),
            "lbm_init": (ctypes.c_int, [P, P, P]),
            "lbm_step": (ctypes.c_int, [P, I32]),
            "lbm_moments": (ctypes.c_int, [P, P, P]),
            "lbm_reduce": (ctypes.c_int, [P, P]),
            "lbm_residual": (ctypes.c_int, [P, P]),
            "lbm_pdfs_export": (ctypes.c_int, [P, P]),
            "lbm_pdfs_import": (ctypes.c_int, [P, P]),
            "lbm_step_count": (I64, [P]),
            "lbm_components": (ctypes.c_int, [I32, P, P, U32, I32, P, P]),
            "lbm_components_device": (ctypes.c_int, [I32, P, P, U32, I32, P, P, P, P]),
            "lbm_components_device_scratch": (I64, [P]),
            "lbm_components_device_noalloc": (ctypes.c_int, [I32, P, P, U32, I32, P, P, P]),
            "lbm_components_noalloc_max_scratch": (I64, []),
            "lbm_project_invariants": (ctypes.c_int, [I32, P, U32, P, I32, ctypes.c_double, I32, P, P, P, P]),
            "lbm_device_copy": (ctypes.c_int, [P, P, ctypes.c_size_t, P]),
            "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "lbm_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, where):
    if rc != LBM_OK:
        detail = lib().lbm_last_error()
        raise LbmError(rc, where, detail.decode() if detail else "")


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def lattice(q):
    """Velocities c[q,3], weights w[q], opposite indices opp[q] of liblbm."""
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q, np.float64)
    opp = np.zeros(q, np.int32)
    _check(lib().lbm_lattice(q, _np_ptr(c), _np_ptr(w), _np_ptr(opp)), "lbm_lattice")
    return c, w, opp


def _periodic_bits(periodic):
    if isinstance(periodic, (int, np.integer)):
        return int(periodic)
    return int(bool(periodic[0])) | (int(bool(periodic[1])) << 1) | (int(bool(periodic[2])) << 2)


def components(solid, lattice=19, axis=-1, periodic=(1, 1, 1)):
    """Host labels (int32, -1 on solid) and count of the fluid components of
    a (nz, ny, nx) mask under the lattice links (axis >= 0: links with
    c_axis != 0 only); lbm_components."""
    m = np.ascontiguousarray(np.asarray(solid).astype(np.uint8))
    if m.ndim == 2:
        m = m[None]
    shape = np.array([m.shape[2], m.shape[1], m.shape[0]], np.int32)
    labels = np.empty(m.shape, np.int32)
    count = ctypes.c_int32()
    _check(lib().lbm_components(int(lattice), _np_ptr(m), _np_ptr(shape), _periodic_bits(periodic), int(axis),
                                _np_ptr(labels), ctypes.byref(count)), "lbm_components")
    return labels, int(count.value)


def device_copy(dst, src, stream=None):
    """lbm_device_copy of src into dst (torch CUDA tensors of equal byte size)."""
    import torch
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("device_copy: sizes differ")
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().lbm_device_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nb,
                                 ctypes.c_void_p(s.cuda_stream)), "lbm_device_copy")


def components_device(solid, lattice=19, axis=-1, periodic=(1, 1, 1), stream=None):
    """Device labels (torch int32, -1 on solid) and count of the fluid
    components of a device uint8 (nz, ny, nx) mask: lbm_components_device,
    the same labels as components()."""
    import torch
    m = solid if solid.dim() == 3 else solid.reshape((1,) + tuple(solid.shape))
    if m.dtype != torch.uint8 or not m.is_contiguous() or not m.is_cuda:
        raise ValueError("solid must be a contiguous uint8 CUDA tensor")
    shape = np.array([m.shape[2], m.shape[1], m.shape[0]], np.int32)
    n_scratch = lib().lbm_components_device_scratch(_np_ptr(shape))
    labels = torch.empty(tuple(m.shape), dtype=torch.int32, device=m.device)
    scratch = torch.empty(max(int(n_scratch), 1), dtype=torch.int32, device=m.device)
    count = ctypes.c_int32()
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().lbm_components_device(int(lattice), ctypes.c_void_p(m.data_ptr()), _np_ptr(shape),
                                       _periodic_bits(periodic), int(axis), ctypes.c_void_p(labels.data_ptr()),
                                       ctypes.byref(count), ctypes.c_void_p(scratch.data_ptr()),
                                       ctypes.c_void_p(s.cuda_stream)), "lbm_components_device")
    return labels, int(count.value)


def components_device_noalloc(solid, labels, lattice=19, axis=-1, periodic=(1, 1, 1), stream=None):
    """lbm_components_device_noalloc: the labels of components_device written
    into the caller's device int32 tensor `labels` (shape of solid), with the
    library's fixed scratch instead of an allocated one; returns the count."""
    import torch
    m = solid if solid.dim() == 3 else solid.reshape((1,) + tuple(solid.shape))
    if m.dtype != torch.uint8 or not m.is_contiguous() or not m.is_cuda:
        raise ValueError("solid must be a contiguous uint8 CUDA tensor")
    if labels.dtype != torch.int32 or not labels.is_contiguous() or labels.numel() != m.numel() or \
            labels.device != m.device:
        raise ValueError("labels must be a contiguous int32 tensor on the mask's device, one entry per node")
    shape = np.array([m.shape[2], m.shape[1], m.shape[0]], np.int32)
    count = ctypes.c_int32()
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().lbm_components_device_noalloc(int(lattice), ctypes.c_void_p(m.data_ptr()), _np_ptr(shape),
                                               _periodic_bits(periodic), int(axis),
                                               ctypes.c_void_p(labels.data_ptr()), ctypes.byref(count),
                                               ctypes.c_void_p(s.cuda_stream)), "lbm_components_device_noalloc")
    return int(count.value)


def components_noalloc_max_scratch():
    """Entries (int32) of the fixed scratch of components_device_noalloc."""
    return int(lib().lbm_components_noalloc_max_scratch())


class Invariants:
    """Component labels of one geometry on the GPU and the scratch for
    lbm_project_invariants.  solid: a host mask (labelled on the host) or a
    device uint8 tensor (labelled on the device, lbm_components_device)."""

    def __init__(self, solid, lattice=19, periodic=(1, 1, 1), device="cuda"):
        import torch
        self.lattice = int(lattice)
        self.periodic = _periodic_bits(periodic)
        if isinstance(solid, torch.Tensor):
            m = solid if solid.dim() == 3 else solid.reshape((1,) + tuple(solid.shape))
            self.shape = tuple(m.shape)
            self.labels, self.count = components_device(m, self.lattice, -1, self.periodic)
        else:
            m = np.asarray(solid)
            if m.ndim == 2:
                m = m[None]
            self.shape = tuple(m.shape)
            lab, self.count = components(m, self.lattice, -1, self.periodic)
            self.labels = torch.from_numpy(lab).to(device)
        n = int(np.prod(self.shape))
        self.scratch = torch.empty(2 * self.count + 6 * n, dtype=torch.float64, device=self.labels.device)

    def project(self, rho, u, rho0=1.0, iterations=8, stream=None):
        """In place on device FP64 rho (nz, ny, nx) and u (3, nz, ny, nx)."""
        import torch
        n = int(np.prod(self.shape))
        if rho.dtype != torch.float64 or u.dtype != torch.float64 or not rho.is_contiguous() or \
                not u.is_contiguous() or rho.numel() != n or u.numel() != 3 * n:
            raise ValueError("rho and u must be contiguous FP64 of %d and %d elements" % (n, 3 * n))
        shape = np.array([self.shape[2], self.shape[1], self.shape[0]], np.int32)
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().lbm_project_invariants(self.lattice, _np_ptr(shape), self.periodic,
                                            ctypes.c_void_p(self.labels.data_ptr()), self.count, float(rho0),
                                            int(iterations), ctypes.c_void_p(rho.data_ptr()),
                                            ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(self.scratch.data_ptr()),
                                            ctypes.c_void_p(s.cuda_stream)), "lbm_project_invariants")


class Tiles:
    """A tiling (lbm_tiles_build / lbm_tiles_concat)."""

    def __init__(self, solid=None, tile=(4, 4, 4), periodic=(1, 1, 1), _handle=None, _parts=None):
        self._h = ctypes.c_void_p()
        self._parts = _parts
        if _handle is not None:
            self._h = _handle
        else:
            solid = np.ascontiguousarray(np.asarray(solid).astype(np.uint8))
            if solid.ndim != 3:
                raise ValueError("solid mask must be (nz, ny, nx)")
            nz, ny, nx = solid.shape
            shape = np.array([nx, ny, nz], np.int32)
            t = np.array(tile, np.int32)
            _check(lib().lbm_tiles_build(_np_ptr(solid), _np_ptr(shape), _np_ptr(t), _periodic_bits(periodic),
                                         ctypes.byref(self._h)), "lbm_tiles_build")
        self.info = self._info()

    @classmethod
    def concat(cls, parts):
        arr = (ctypes.c_void_p * len(parts))(*[p._h.value for p in parts])
        h = ctypes.c_void_p()
        _check(lib().lbm_tiles_concat(arr, len(parts), ctypes.byref(h)), "lbm_tiles_concat")
        return cls(_handle=h, _parts=list(parts))

    def _info(self):
        i = TilesInfo()
        _check(lib().lbm_tiles_info(self._h, ctypes.byref(i)), "lbm_tiles_info")
        return dict(shape=tuple(i.shape), grid=tuple(i.grid), tile=tuple(i.tile), tgrid=tuple(i.tgrid),
                    periodic=i.periodic, words=i.words, n_samples=i.n_samples, n_tiles=i.n_tiles,
                    n_ftiles=i.n_ftiles, n_fluid=i.n_fluid, n_nodes=i.n_nodes, phi=i.phi, phi_t=i.phi_t,
                    tiles_ratio=i.tiles_ratio, alpha_m=i.alpha_m)

    def export(self):
        i = self.info
        tm = np.zeros(i["n_tiles"], np.int32)
        co = np.zeros(3 * i["n_ftiles"], np.int32)
        nb = np.zeros(27 * i["n_ftiles"], np.int32)
        fl = np.zeros(i["words"] * i["n_ftiles"], np.uint64)
        _check(lib().lbm_tiles_export(self._h, _np_ptr(tm), _np_ptr(co), _np_ptr(nb), _np_ptr(fl)),
               "lbm_tiles_export")
        return dict(tile_map=tm, tile_coord=co, nbr=nb, fluid=fl)

    def __del__(self):
        try:
            if self._h and self._h.value:
                lib().lbm_tiles_free(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass


def make_params(lattice=19, storage="f64", tau=0.7, g=(0.0, 0.0, 0.0), rho0=1.0, f16_scale_log2=20,
                tiles_per_block=0, tile_order="morton", step_kernel="auto", store_policy="auto", persistent=0,
                graph_steps=0, model="quasi-compressible", pattern="two-copy", collision="bgk", mrt_rates=None):
    """mrt_rates: (s_e, s_eps, s_q, s_pi, s_m) of the MRT collision; None or 0 entries take the published
    defaults of the lattice."""
    p = Params()
    p.lattice = lattice
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.tau = float(tau)
    for k in range(3):
        p.g[k] = float(g[k])
    p.rho0 = float(rho0)
    p.f16_scale_log2 = int(f16_scale_log2)
    p.tiles_per_block = int(tiles_per_block)
    p.tile_order = ORDER[tile_order] if isinstance(tile_order, str) else int(tile_order)
    p.step_kernel = KERNEL[step_kernel] if isinstance(step_kernel, str) else int(step_kernel)
    p.store_policy = STORE_POLICY[store_policy] if isinstance(store_policy, str) else int(store_policy)
    p.persistent = int(bool(persistent))
    p.graph_steps = int(graph_steps)
    p.model = MODEL[model] if isinstance(model, str) else int(model)
    p.pattern = PATTERN[pattern] if isinstance(pattern, str) else int(pattern)
    p.collision = COLLISION[collision] if isinstance(collision, str) else int(collision)
    for k, r in enumerate(mrt_rates if mrt_rates is not None else ()):
        p.mrt_rates[k] = float(r)
    return p


def workspace_bytes(tiles, **params):
    n = ctypes.c_size_t()
    p = make_params(**params)
    _check(lib().lbm_workspace_bytes(tiles._h, ctypes.byref(p), ctypes.byref(n)), "lbm_workspace_bytes")
    return n.value


class Solver:
    """A solver on one tiling; device memory and stream come from torch."""

    def __init__(self, tiles, lattice=19, storage="f64", tau=0.7, g=(0.0, 0.0, 0.0), rho0=1.0, f16_scale_log2=20,
                 tiles_per_block=0, tile_order="morton", step_kernel="auto", store_policy="auto", persistent=0,
                 graph_steps=0, model="quasi-compressible", pattern="two-copy", collision="bgk", mrt_rates=None,
                 device="cuda", stream=None, workspace=None):
        """workspace: optional caller-owned device tensor (uint8, at least
        workspace_bytes(tiles, ...) long, 256-byte aligned); by default the
        solver allocates its own."""
        import torch

        self.torch = torch
        self.tiles = tiles
        self.q = lattice
        self.params = make_params(lattice, storage, tau, g, rho0, f16_scale_log2, tiles_per_block, tile_order,
                                  step_kernel, store_policy, persistent, graph_steps, model, pattern, collision,
                                  mrt_rates)
        self.device = torch.device(device)
        n = ctypes.c_size_t()
        _check(lib().lbm_workspace_bytes(tiles._h, ctypes.byref(self.params), ctypes.byref(n)),
               "lbm_workspace_bytes")
        if workspace is None:
            self.workspace = torch.empty(max(n.value, 256), dtype=torch.uint8, device=self.device)
        else:
            if workspace.dtype != torch.uint8 or workspace.numel() < n.value or not workspace.is_contiguous():
                raise ValueError("workspace must be contiguous uint8 of at least %d bytes" % n.value)
            self.workspace = workspace
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        _check(lib().lbm_create(tiles._h, ctypes.byref(self.params), ctypes.c_void_p(self.workspace.data_ptr()),
                                n.value, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)),
               "lbm_create")
        info = tiles.info
        self.n_samples = info["n_samples"]
        self.dense_shape = (info["shape"][2], info["shape"][1], info["shape"][0]) if self.n_samples == 1 else None
        self.n_nodes = info["n_nodes"]

    # shapes of dense fields
    def _scalar_shape(self):
        return self.dense_shape if self.dense_shape else (self.n_nodes,)

    def _vec_shape(self):
        return (3,) + self.dense_shape if self.dense_shape else (3 * self.n_nodes,)

    def _pdf_shape(self):
        return (self.q,) + self.dense_shape if self.dense_shape else (self.q * self.n_nodes,)

    def _dev(self, t, shape):
        torch = self.torch
        t = t.to(device=self.device, dtype=torch.float64).contiguous()
        if t.numel() != int(np.prod(shape)):
            raise ValueError("expected %d elements, got %d" % (int(np.prod(shape)), t.numel()))
        return t

    def init(self, rho=None, u=None):
        r = None if rho is None else self._dev(rho, self._scalar_shape())
        v = None if u is None else self._dev(u, self._vec_shape())
        _check(lib().lbm_init(self._h, ctypes.c_void_p(r.data_ptr()) if r is not None else None,
                              ctypes.c_void_p(v.data_ptr()) if v is not None else None), "lbm_init")
        self._keep = (r, v)  # alive until the stream has consumed them
        self.stream.synchronize()
        self._keep = None

    def step(self, n=1):
        _check(lib().lbm_step(self._h, int(n)), "lbm_step")

    def moments(self):
        torch = self.torch
        rho = torch.empty(self._scalar_shape(), dtype=torch.float64, device=self.device)
        u = torch.empty(self._vec_shape(), dtype=torch.float64, device=self.device)
        _check(lib().lbm_moments(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(u.data_ptr())),
               "lbm_moments")
        return rho, u

    def reduce(self):
        out = np.zeros(4 * self.n_samples)
        _check(lib().lbm_reduce(self._h, _np_ptr(out)), "lbm_reduce")
        return out.reshape(self.n_samples, 4)

    def residual(self):
        out = np.zeros(self.n_samples)
        _check(lib().lbm_residual(self._h, _np_ptr(out)), "lbm_residual")
        return out

    def pdfs_export(self):
        torch = self.torch
        f = torch.empty(self._pdf_shape(), dtype=torch.float64, device=self.device)
        _check(lib().lbm_pdfs_export(self._h, ctypes.c_void_p(f.data_ptr())), "lbm_pdfs_export")
        return f

    def pdfs_import(self, f):
        f = self._dev(f, self._pdf_shape())
        _check(lib().lbm_pdfs_import(self._h, ctypes.c_void_p(f.data_ptr())), "lbm_pdfs_import")
        self.stream.synchronize()

    def set_sample_force(self, g):
        g = np.ascontiguousarray(np.asarray(g, np.float64).reshape(-1))
        if g.size != 3 * self.n_samples:
            raise ValueError("need 3 values per sample")
        _check(lib().lbm_set_sample_force(self._h, _np_ptr(g)), "lbm_set_sample_force")

    def set_lid(self, axis, side=1, u=(0.0, 0.0, 0.0)):
        """Moving wall on the face of non-periodic `axis` beyond the last node (side 1) or before the first
        (side 0), velocity u; axis=None removes it."""
        if axis is None:
            _check(lib().lbm_set_lid(self._h, -1, 0, None), "lbm_set_lid")
            return
        uu = np.ascontiguousarray(np.asarray(u, np.float64).reshape(3))
        _check(lib().lbm_set_lid(self._h, int(axis), int(side), _np_ptr(uu)), "lbm_set_lid")

    def set_active(self, active):
        a = np.ascontiguousarray(np.asarray(active).astype(np.uint8).reshape(-1))
        if a.size != self.n_samples:
            raise ValueError("need one flag per sample")
        _check(lib().lbm_set_active(self._h, _np_ptr(a)), "lbm_set_active")

    def run_to_steady(self, tol=1e-6, check_every=100, max_steps=1_000_000, batch_deactivate=True, progress=None):
        """Step until every sample's residual (velocity change over
        ``check_every`` steps, relative) is below ``tol``.  For batches,
        converged samples are taken out of the active tile list.  Returns
        (steps taken per sample, final residuals).  ``progress``: a callable
        given (steps, number converged, max residual of the rest) about every
        20 s."""
        import time
        n = self.n_samples
        last = time.perf_counter()
        done = np.zeros(n, bool)
        steps_at = np.full(n, -1, np.int64)
        res = np.full(n, np.inf)
        self.residual()  # reference velocity
        taken = 0
        while taken < max_steps and not done.all():
            self.step(check_every)
            taken += check_every
            res = self.residual()
            newly = (~done) & (res < tol)
            if newly.any():
                steps_at[newly] = taken
                done |= newly
                if batch_deactivate and n > 1 and not done.all():
                    self.set_active(~done)
            if progress is not None and time.perf_counter() - last > 20:
                last = time.perf_counter()
                progress(taken, int(done.sum()), float(res[~done].max()) if (~done).any() else 0.0)
        steps_at[~done] = -1
        return steps_at, res

    @property
    def step_count(self):
        return lib().lbm_step_count(self._h)

    def synchronize(self):
        self.stream.synchronize()

    def __del__(self):
        try:
            if self._h and self._h.value:
                lib().lbm_destroy(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass
