"""ctypes binding of liblumiq.so (include/lumiq.h).

Argument marshalling only: torch tensors supply device memory and streams,
every step of the query runs in the library's HIP kernels.  The binding fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblumiq.so")

LQ_OK = 0
LQ_F32, LQ_F16, LQ_BF16 = 0, 1, 2
LQ_LINEAR, LQ_EXP = 0, 1
LQ_NO_EARLY_TERM, LQ_FP64_ACCUM, LQ_NO_SIGMA_SKIP, LQ_TRACE_PRUNED = 1, 2, 4, 8

STORAGE = {"f32": LQ_F32, "f16": LQ_F16, "bf16": LQ_BF16}
MODEL = {"linear": LQ_LINEAR, "exp": LQ_EXP}
STATUS = {0: "LQ_OK", -1: "LQ_ERR_INVALID_ARG", -2: "LQ_ERR_FORMAT", -3: "LQ_ERR_OOM",
          -4: "LQ_ERR_HIP", -5: "LQ_ERR_UNSUPPORTED", -6: "LQ_ERR_STATE", -7: "LQ_ERR_IO"}


class LumiqError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class OctreeDesc(C.Structure):
    _fields_ = [("max_depth", C.c_int32), ("sh_degree", C.c_int32), ("n_nodes", C.c_int32),
                ("n_leaves", C.c_int32), ("l_max", C.c_float), ("sigma_min", C.c_float),
                ("alpha_max", C.c_float), ("child", C.c_void_p), ("sigma", C.c_void_p),
                ("sh", C.c_void_p)]


class FieldDesc(C.Structure):
    _fields_ = [("n_blobs", C.c_int32), ("n_shells", C.c_int32), ("sh_degree", C.c_int32),
                ("reserved", C.c_int32), ("blobs", C.c_void_p), ("blob_sh", C.c_void_p),
                ("shells", C.c_void_p), ("shell_half_width", C.c_double),
                ("log_density_base", C.c_double), ("sigma_max", C.c_double), ("l_max", C.c_double)]


_lock = threading.Lock()
_lib = None


def lib():
    """Load liblumiq.so (raises if it is missing)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
            # PyTorch ships a HIP runtime of its own and puts it in the process's
            # global symbol scope when imported.  Importing it before the library
            # is loaded binds the library's HIP calls to that same runtime, the one
            # that owns torch's memory and streams.  Loaded the other way round, the
            # library would start the system runtime first, and torch's runtime,
            # started second, finds no GPU.
            import torch  # noqa: F401
            L = C.CDLL(LIB_PATH)
            vp, i64, i32, u32 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32
            L.lq_last_error.restype = C.c_char_p
            L.lq_version.restype = C.c_char_p
            L.lq_load_octree_desc.argtypes = [C.POINTER(OctreeDesc), C.c_int, C.c_int, C.POINTER(vp)]
            L.lq_load_octree.argtypes = [C.c_char_p, C.c_int, C.c_int, C.POINTER(vp)]
            L.lq_free_octree.argtypes = [vp]
            L.lq_free_octree.restype = None
            L.lq_octree_info.argtypes = [vp] + [C.c_void_p] * 6
            L.lq_query_radiance.argtypes = [vp, vp, vp, i64, vp, vp, C.c_int, u32, vp]
            L.lq_query_trace.argtypes = [vp, vp, vp, i64, vp, vp, C.c_int, u32,
                                         vp, vp, vp, vp, vp, vp, i32, vp]
            L.lq_query_radiance_image.argtypes = [vp, vp, vp, i32, i32, vp, vp, C.c_int, u32, vp]
            L.lq_proxy_irradiance.argtypes = [vp, vp, vp, i64, vp, i32, vp, C.c_int, vp, vp, vp]
            L.lq_distill_leaves.argtypes = [C.POINTER(FieldDesc), i32, C.c_float, i32, C.c_uint64, C.c_int,
                                            i64, vp, vp, vp, C.POINTER(i64), vp]
            L.lq_octree_from_leaves.argtypes = [i32, i32, vp, vp, vp, i64, C.c_float, C.c_float, C.c_float,
                                                C.c_int, C.c_int, C.POINTER(vp)]
            L.lq_octree_download.argtypes = [vp, vp, vp, vp]
            L.lq_proxy_guide.argtypes = [vp, i32, i32, i32, vp, C.c_int, vp, vp]
            L.lq_proxy_irradiance_guided.argtypes = [vp, vp, vp, i64, vp, i32, vp, i32, i32, C.c_float, vp, C.c_int,
                                                     vp, vp, vp]
            for name in ("lq_load_octree_desc", "lq_load_octree", "lq_octree_info",
                         "lq_query_radiance", "lq_query_trace", "lq_query_radiance_image",
                         "lq_proxy_irradiance", "lq_distill_leaves", "lq_octree_from_leaves",
                         "lq_octree_download", "lq_proxy_guide", "lq_proxy_irradiance_guided"):
                getattr(L, name).restype = C.c_int
            _lib = L
    return _lib


def check(status: int) -> None:
    if status != LQ_OK:
        raise LumiqError(status, lib().lq_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Octree:
    """A plenoctree resident on one GPU.

    tree: an object with depth, sh_degree, l_max, sigma_min, alpha_max,
    child [n_nodes, 8] int32, sigma [n_leaves] float32, sh [n_leaves, 3, K]
    float32 (e.g. inputs.Tree), or a path to an LQOT file.
    """

    def __init__(self, tree, storage: str = "f32", device: int = 0):
        self.handle = C.c_void_p()
        self.device = device
        self.storage = storage
        st = STORAGE[storage]
        if isinstance(tree, (str, os.PathLike)):
            check(lib().lq_load_octree(os.fsencode(tree), st, device, C.byref(self.handle)))
        else:
            child = np.ascontiguousarray(tree.child, dtype=np.int32)
            sigma = np.ascontiguousarray(tree.sigma, dtype=np.float32)
            sh = np.ascontiguousarray(tree.sh, dtype=np.float32)
            desc = OctreeDesc(int(tree.depth), int(tree.sh_degree), child.shape[0], sigma.shape[0],
                              float(tree.l_max), float(tree.sigma_min), float(tree.alpha_max),
                              child.ctypes.data, sigma.ctypes.data if sigma.size else None,
                              sh.ctypes.data if sh.size else None)
            check(lib().lq_load_octree_desc(C.byref(desc), st, device, C.byref(self.handle)))

    @classmethod
    def _adopt(cls, handle, storage: str, device: int) -> "Octree":
        self = cls.__new__(cls)
        self.handle = handle
        self.device = device
        self.storage = storage
        return self

    def download(self) -> dict:
        """The tree's tables as stored: child [n_nodes, 8] int32, sigma
        [n_leaves] and sh [n_leaves, 3, K] float32 (numpy)."""
        inf = self.info()
        K = (inf["sh_degree"] + 1) ** 2
        child = np.zeros((inf["n_nodes"], 8), np.int32)
        sigma = np.zeros(inf["n_leaves"], np.float32)
        sh = np.zeros((inf["n_leaves"], 3, K), np.float32)
        check(lib().lq_octree_download(self.handle, child.ctypes.data, sigma.ctypes.data if sigma.size else None,
                                       sh.ctypes.data if sh.size else None))
        return {"child": child, "sigma": sigma, "sh": sh}

    def info(self) -> dict:
        v = [C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()]
        check(lib().lq_octree_info(self.handle, *[C.byref(x) for x in v]))
        keys = ("device_bytes", "n_nodes", "n_leaves", "max_depth", "sh_degree", "storage")
        return {k: x.value for k, x in zip(keys, v)}

    def free(self) -> None:
        if self.handle:
            lib().lq_free_octree(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def query(self, origins, dirs, model: str = "linear", flags: int = 0, rgb=None,
              alpha=None, want_alpha: bool = True, stream=None):
        """Emission query.  origins/dirs: float32 [n, 3] CUDA tensors.
        Returns (rgb [n, 3], alpha [n] or None)."""
        import torch
        n = origins.shape[0]
        if rgb is None:
            rgb = torch.empty((n, 3), dtype=torch.float32, device=origins.device)
        if alpha is None and want_alpha:
            alpha = torch.empty((n,), dtype=torch.float32, device=origins.device)
        check(lib().lq_query_radiance(self.handle, _ptr(origins), _ptr(dirs), n, _ptr(rgb),
                                      _ptr(alpha), MODEL[model], flags, _stream(stream)))
        return rgb, alpha

    def query_image(self, origins, dirs, width: int, height: int, model: str = "linear",
                    flags: int = 0, rgb=None, alpha=None, want_alpha: bool = True, stream=None):
        """Emission query of a camera batch: origins/dirs float32 [height * width, 3]
        CUDA tensors in row-major pixel order.  Same results as query(); the
        device takes the rays up in 8 x 8 pixel tiles.  Returns (rgb, alpha)."""
        import torch
        n = width * height
        if origins.shape[0] != n or dirs.shape[0] != n:
            raise ValueError(f"expected {n} rays for a {width} x {height} image")
        if rgb is None:
            rgb = torch.empty((n, 3), dtype=torch.float32, device=origins.device)
        if alpha is None and want_alpha:
            alpha = torch.empty((n,), dtype=torch.float32, device=origins.device)
        check(lib().lq_query_radiance_image(self.handle, _ptr(origins), _ptr(dirs), width, height,
                                            _ptr(rgb), _ptr(alpha), MODEL[model], flags,
                                            _stream(stream)))
        return rgb, alpha

    def proxy_irradiance(self, points, normals, u, background=None, model: str = "linear",
                         want_terms: bool = False, irradiance=None, stream=None):
        """Irradiance [n, 3] at shading points from the light leaving the proxy
        (emission plus the background through the luminaire), estimated with
        u.shape[1] uniform proxy samples per point.  points/normals: float32
        [n, 3], u: float32 [n, S, 3] CUDA tensors.  Returns (irradiance,
        terms [n, S, 3] or None)."""
        import torch
        n, S = u.shape[0], u.shape[1]
        if points.shape[0] != n or normals.shape[0] != n:
            raise ValueError("points, normals and u disagree on the number of points")
        if irradiance is None:
            irradiance = torch.empty((n, 3), dtype=torch.float32, device=points.device)
        terms = torch.empty((n, S, 3), dtype=torch.float32, device=points.device) if want_terms else None
        bg = (C.c_float * 3)(*background) if background is not None else None
        check(lib().lq_proxy_irradiance(self.handle, _ptr(points), _ptr(normals), n, _ptr(u), S, bg,
                                        MODEL[model], _ptr(irradiance), _ptr(terms), _stream(stream)))
        return irradiance, terms

    def proxy_guide(self, grid: int, u_probe, model: str = "linear", weights=None, stream=None,
                    dir_res: int = 1):
        """Guide weights [6 grid^2 dir_res^2] (cell-major) of the proxy's
        cells from probe rays (u_probe: float32 [6 grid^2, R, 5] CUDA tensor),
        one per direction bin.  dir_res = 1 averages over directions; 2 x 2
        bins with a few hundred probes per cell gave the lowest estimator
        variance on the benchmark's floor (finer bins need more probes)."""
        import torch
        n_cells = 6 * grid * grid
        if u_probe.shape[0] != n_cells or u_probe.shape[2] != 5:
            raise ValueError(f"u_probe must be [{n_cells}, R, 5]")
        if weights is None:
            weights = torch.empty((n_cells * dir_res * dir_res,), dtype=torch.float32, device=u_probe.device)
        check(lib().lq_proxy_guide(self.handle, grid, dir_res, u_probe.shape[1], _ptr(u_probe), MODEL[model],
                                   _ptr(weights), _stream(stream)))
        return weights

    def proxy_irradiance_guided(self, points, normals, u, weights, grid: int, defensive: float = 0.25,
                                background=None, model: str = "linear", want_terms: bool = False,
                                irradiance=None, stream=None, dir_res: int = 1):
        """proxy_irradiance with the samples' cells drawn from a guide
        (weights [6 grid^2 dir_res^2], as proxy_guide writes them)."""
        import torch
        n, S = u.shape[0], u.shape[1]
        if irradiance is None:
            irradiance = torch.empty((n, 3), dtype=torch.float32, device=points.device)
        terms = torch.empty((n, S, 3), dtype=torch.float32, device=points.device) if want_terms else None
        bg = (C.c_float * 3)(*background) if background is not None else None
        check(lib().lq_proxy_irradiance_guided(self.handle, _ptr(points), _ptr(normals), n, _ptr(u), S,
                                               _ptr(weights), grid, dir_res, defensive, bg, MODEL[model],
                                               _ptr(irradiance), _ptr(terms), _stream(stream)))
        return irradiance, terms

    def trace(self, origins, dirs, model: str = "linear", flags: int = 0, max_ids: int = 0,
              stream=None) -> dict:
        """Validation query: radiance plus per-ray leaf records."""
        import torch
        n = origins.shape[0]
        dev = origins.device
        out = {
            "rgb": torch.empty((n, 3), dtype=torch.float32, device=dev),
            "alpha": torch.empty((n,), dtype=torch.float32, device=dev),
            "count": torch.empty((n,), dtype=torch.int32, device=dev),
            "hash": torch.empty((n,), dtype=torch.int64, device=dev),
            "term_idx": torch.empty((n,), dtype=torch.int32, device=dev),
            "n_comp": torch.empty((n,), dtype=torch.int32, device=dev),
            "n_steps": torch.empty((n,), dtype=torch.int32, device=dev),
        }
        ids = torch.zeros((n, max_ids), dtype=torch.int32, device=dev) if max_ids > 0 else None
        check(lib().lq_query_trace(self.handle, _ptr(origins), _ptr(dirs), n, _ptr(out["rgb"]),
                                   _ptr(out["alpha"]), MODEL[model], flags, _ptr(out["count"]),
                                   _ptr(out["hash"]), _ptr(out["term_idx"]), _ptr(out["n_comp"]),
                                   _ptr(out["n_steps"]), _ptr(ids), max_ids, _stream(stream)))
        if ids is not None:
            out["leaf_ids"] = ids
        return out


def field_desc(p: dict):
    """lq_field_desc from field parameters (centres [nb, 3], radii, amps,
    emission [nb, 3], hi [nb, 3, K-1], shells [ns, 4], shell_half_width,
    log_base, sigma_max, l_max, sh_degree).  Returns (desc, arrays kept
    alive)."""
    nb = len(p["radii"])
    blobs = np.ascontiguousarray(np.concatenate([np.asarray(p["centres"], np.float64).reshape(nb, 3),
                                                 np.asarray(p["radii"], np.float64).reshape(nb, 1),
                                                 np.asarray(p["amps"], np.float64).reshape(nb, 1),
                                                 np.asarray(p["emission"], np.float64).reshape(nb, 3)], axis=1))
    hi = np.ascontiguousarray(np.asarray(p["hi"], np.float64).reshape(-1))
    shells = np.ascontiguousarray(np.asarray(p["shells"], np.float64).reshape(-1, 4))
    desc = FieldDesc(nb, shells.shape[0], int(p["sh_degree"]), 0, blobs.ctypes.data,
                     hi.ctypes.data if hi.size else None, shells.ctypes.data if shells.size else None,
                     float(p["shell_half_width"]), float(p["log_base"]), float(p["sigma_max"]), float(p["l_max"]))
    return desc, (blobs, hi, shells)


def distill_leaves(params: dict, depth: int, prune_sigma: float = 0.01, n_samples: int = 256, seed: int = 0,
                   device: int = 0, stream=None):
    """Plenoctree distillation of a continuous field (Sec. 5): returns the
    kept voxels' Morton codes (int32 view of the uint32 codes, ascending),
    mean densities and mean SH coefficients as CUDA tensors."""
    import torch
    L = lib()
    desc, keep = field_desc(params)
    n = C.c_int64()
    check(L.lq_distill_leaves(C.byref(desc), depth, prune_sigma, n_samples, seed, device, 0, None, None, None,
                              C.byref(n), _stream(stream)))
    K = (int(params["sh_degree"]) + 1) ** 2
    dev = torch.device("cuda", device)
    codes = torch.empty((max(n.value, 1),), dtype=torch.int32, device=dev)
    sigma = torch.empty((max(n.value, 1),), dtype=torch.float32, device=dev)
    sh = torch.empty((max(n.value, 1), 3, K), dtype=torch.float32, device=dev)
    check(L.lq_distill_leaves(C.byref(desc), depth, prune_sigma, n_samples, seed, device, n.value, _ptr(codes),
                              _ptr(sigma), _ptr(sh), C.byref(n), _stream(stream)))
    del keep
    return codes[: n.value], sigma[: n.value], sh[: n.value]


def octree_from_leaves(depth: int, sh_degree: int, codes, sigma, sh, l_max: float = 2048.0,
                       sigma_min: float = 0.1, alpha_max: float = 0.9, storage: str = "f32",
                       device: int = 0) -> Octree:
    """An Octree (device-built child table) from leaves at max depth."""
    h = C.c_void_p()
    n = codes.shape[0]
    check(lib().lq_octree_from_leaves(depth, sh_degree, _ptr(codes) if n else None, _ptr(sigma) if n else None,
                                      _ptr(sh) if n else None, n, l_max, sigma_min, alpha_max, STORAGE[storage],
                                      device, C.byref(h)))
    return Octree._adopt(h, storage, device)


def version() -> str:
    return lib().lq_version().decode()


# ------------------------------------------------------------------ surrogate
class MlpConfig(C.Structure):
    _fields_ = [("n_freq", C.c_int32), ("hidden", C.c_int32), ("n_hidden_layers", C.c_int32)]


class TrainConfig(C.Structure):
    _fields_ = [("steps", C.c_int32), ("total_steps", C.c_int32), ("batch", C.c_int32),
                ("lr0", C.c_float), ("lr1", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


_mlp_ready = False


def _mlp_lib():
    global _mlp_ready
    L = lib()
    if not _mlp_ready:
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.lq_mlp_create.argtypes = [C.POINTER(MlpConfig), C.c_uint64, C.c_int, C.POINTER(vp)]
        L.lq_mlp_free.argtypes = [vp]
        L.lq_mlp_free.restype = None
        L.lq_mlp_num_params.restype = C.c_int32
        L.lq_mlp_get_params.argtypes = [vp, vp]
        L.lq_mlp_set_params.argtypes = [vp, vp]
        L.lq_mlp_train.argtypes = [vp, vp, vp, vp, i64, C.POINTER(TrainConfig), vp, vp]
        L.lq_mlp_grad.argtypes = [vp, vp, vp, vp, i64, vp, C.POINTER(C.c_float), vp]
        L.lq_mlp_forward.argtypes = [vp, vp, vp, i64, vp, vp]
        L.lq_mlp_build_trust.argtypes = [vp, vp, vp, vp, i64, C.c_float, vp]
        L.lq_mlp_trust_map.argtypes = [vp, vp, C.POINTER(i32)]
        L.lq_mlp_infer.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
        L.lq_mlp_save.argtypes = [vp, C.c_char_p]
        L.lq_mlp_load.argtypes = [C.c_char_p, C.c_int, C.POINTER(vp)]
        L.lq_query_radiance_multi.argtypes = [C.POINTER(vp), i32, vp, vp, vp, vp, vp, C.c_int,
                                              C.c_uint32, vp]
        for name in ("lq_mlp_create", "lq_mlp_get_params", "lq_mlp_set_params", "lq_mlp_train",
                     "lq_mlp_grad", "lq_mlp_forward", "lq_mlp_build_trust", "lq_mlp_trust_map",
                     "lq_mlp_infer", "lq_mlp_save", "lq_mlp_load", "lq_query_radiance_multi"):
            getattr(L, name).restype = C.c_int
        _mlp_ready = True
    return L


class Surrogate:
    """The learned surrogate (Fourier features + 4 x 64 MLP) on one GPU."""

    def __init__(self, seed: int = 31, device: int = 0, path: str | None = None):
        L = _mlp_lib()
        self.handle = C.c_void_p()
        self.device = device
        if path is not None:
            check(L.lq_mlp_load(os.fsencode(path), device, C.byref(self.handle)))
        else:
            cfg = MlpConfig(10, 64, 4)
            check(L.lq_mlp_create(C.byref(cfg), seed, device, C.byref(self.handle)))
        self.n_params = int(L.lq_mlp_num_params())

    def free(self):
        if self.handle:
            _mlp_lib().lq_mlp_free(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        check(_mlp_lib().lq_mlp_get_params(self.handle, out.ctypes.data))
        return out

    def set_params(self, theta) -> None:
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        assert theta.shape == (self.n_params,)
        check(_mlp_lib().lq_mlp_set_params(self.handle, theta.ctypes.data))

    def train(self, origins, dirs, rgb, steps: int, total_steps: int | None = None,
              batch: int = 65536, lr0: float = 5e-4, lr1: float = 5e-6, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, log: bool = True, stream=None):
        cfg = TrainConfig(steps, total_steps or steps, batch, lr0, lr1, beta1, beta2, eps)
        losses = np.zeros(max(steps, 1), np.float32) if log else None
        check(_mlp_lib().lq_mlp_train(self.handle, _ptr(origins), _ptr(dirs), _ptr(rgb),
                                      origins.shape[0], C.byref(cfg),
                                      losses.ctypes.data if log else None, _stream(stream)))
        return losses[:steps] if log else None

    def grad(self, origins, dirs, rgb, stream=None):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=origins.device)
        loss = C.c_float()
        check(_mlp_lib().lq_mlp_grad(self.handle, _ptr(origins), _ptr(dirs), _ptr(rgb),
                                     origins.shape[0], _ptr(g), C.byref(loss), _stream(stream)))
        return float(loss.value), g

    def forward(self, origins, dirs, rgb=None, stream=None):
        import torch
        n = origins.shape[0]
        if rgb is None:
            rgb = torch.empty((n, 3), dtype=torch.float32, device=origins.device)
        check(_mlp_lib().lq_mlp_forward(self.handle, _ptr(origins), _ptr(dirs), n, _ptr(rgb),
                                        _stream(stream)))
        return rgb

    def build_trust(self, origins, dirs, rgb_ref, max_rel_err: float = 0.01, stream=None):
        check(_mlp_lib().lq_mlp_build_trust(self.handle, _ptr(origins), _ptr(dirs), _ptr(rgb_ref),
                                            origins.shape[0], max_rel_err, _stream(stream)))

    def trust_map(self) -> np.ndarray | None:
        nb = C.c_int32()
        check(_mlp_lib().lq_mlp_trust_map(self.handle, None, C.byref(nb)))
        if nb.value == 0:
            return None
        out = np.zeros(nb.value, np.uint8)
        check(_mlp_lib().lq_mlp_trust_map(self.handle, out.ctypes.data, C.byref(nb)))
        return out

    def infer(self, origins, dirs, fallback: "Octree | None", rgb=None, want_used: bool = True,
              stream=None):
        import torch
        n = origins.shape[0]
        if rgb is None:
            rgb = torch.empty((n, 3), dtype=torch.float32, device=origins.device)
        used = torch.empty((n,), dtype=torch.uint8, device=origins.device) if want_used else None
        check(_mlp_lib().lq_mlp_infer(self.handle, fallback.handle if fallback else None,
                                      _ptr(origins), _ptr(dirs), n, _ptr(rgb), _ptr(used),
                                      _stream(stream)))
        return rgb, used

    def save(self, path: str) -> None:
        check(_mlp_lib().lq_mlp_save(self.handle, os.fsencode(path)))


def query_multi(trees, offsets, origins, dirs, model: str = "linear", flags: int = 0,
                rgb=None, alpha=None, stream=None):
    """One launch over several luminaires: rays [offsets[k], offsets[k+1])
    query trees[k] (Octree objects)."""
    import torch
    L = _mlp_lib()
    n = origins.shape[0]
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    assert offs.shape == (len(trees) + 1,) and offs[-1] == n
    handles = (C.c_void_p * len(trees))(*[t.handle.value for t in trees])
    if rgb is None:
        rgb = torch.empty((n, 3), dtype=torch.float32, device=origins.device)
    if alpha is None:
        alpha = torch.empty((n,), dtype=torch.float32, device=origins.device)
    check(L.lq_query_radiance_multi(handles, len(trees), offs.ctypes.data, _ptr(origins), _ptr(dirs),
                                    _ptr(rgb), _ptr(alpha), MODEL[model], flags, _stream(stream)))
    return rgb, alpha
