"""Python front end of the fpt C ABI.

Torch provides device memory and the current HIP stream; all transport work
runs in libfpt.so.  Scenes and runs are plain dictionaries (see the
`workloads` module for the schema).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi
from ._abi import check, lib

TALLY_NAMES = _abi.TALLY_NAMES
EXIT_NAMES = _abi.EXIT_NAMES


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _require_cuda(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")


class Scene:
    """A scene uploaded to the current device (fpt_scene_create)."""

    def __init__(self, desc: dict):
        self.desc = desc
        # the differentiable parameters the scene's tables currently hold:
        # [conc per (medium, dye slot)] + [QY per dye] + [sigma_s per medium]
        self.theta = np.array([c for m in desc["media"] for _, c in m["dyes"]] +
                              [d["qy"] for d in desc["dyes"]] +
                              [m["sigma_s"] for m in desc["media"]], dtype=np.float64)
        self._d = _abi.scene_desc(desc)
        h = C.c_void_p()
        check(lib().fpt_scene_create(C.byref(self._d), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().fpt_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def film_shape(self, batches=1):
        dims = (C.c_int64 * 5)()
        nd = C.c_int32()
        check(lib().fpt_film_shape(self._h, batches, dims, C.byref(nd)))
        return tuple(dims[: nd.value])

    @property
    def n_params(self):
        n = lib().fpt_grad_param_count(self._h)
        if n < 0:
            check(n)
        return n

    def set_params(self, conc=None, qy=None, sigma_s=None):
        """fpt_scene_set_params on the current stream: renders enqueued after
        this call see the new parameters."""
        def arr(x):
            return None if x is None else np.ascontiguousarray(x, dtype=np.float64)
        c, q, s = arr(conc), arr(qy), arr(sigma_s)
        check(lib().fpt_scene_set_params(
            self._h, None if c is None else c.ctypes.data, None if q is None else q.ctypes.data,
            None if s is None else s.ctypes.data, _stream()))
        nc = sum(len(m["dyes"]) for m in self.desc["media"])
        nd = len(self.desc["dyes"])
        th = self.theta.copy()
        for part, lo, n in ((c, 0, nc), (q, nc, nd), (s, nc + nd, len(self.desc["media"]))):
            if part is not None:
                th[lo:lo + n] = part[:n]
        self.theta = th

    def set_tune(self, block_threads=0, blocks_per_cu=0, refill_lanes=0, chunk_paths=0,
                 block_min_vertices=0, block_segments=0, wide_rounds=0):
        t = _abi.Tune(block_threads, blocks_per_cu, refill_lanes, chunk_paths,
                      block_min_vertices, block_segments, wide_rounds)
        check(lib().fpt_scene_set_tune(self._h, C.byref(t)))

    def set_timing(self, enable=True):
        """fpt_scene_set_timing: record launch events in later renders."""
        check(lib().fpt_scene_set_timing(self._h, 1 if enable else 0))

    def timing(self):
        """fpt_scene_timing: (renders, mean transport ms, mean deferred-connection ms)."""
        n, t, d = C.c_int32(), C.c_float(), C.c_float()
        check(lib().fpt_scene_timing(self._h, C.byref(n), C.byref(t), C.byref(d)))
        return n.value, t.value, d.value

    def timing_each(self, cap=4096):
        """fpt_scene_timing_each: (transport ms, deferred ms) arrays, one entry
        per timed render."""
        t = np.zeros(cap, np.float32)
        d = np.zeros(cap, np.float32)
        n = C.c_int32()
        check(lib().fpt_scene_timing_each(self._h, cap, C.byref(n), t.ctypes.data, d.ctypes.data))
        k = min(n.value, cap)
        return t[:k].astype(np.float64), d[:k].astype(np.float64)

    def tables(self):
        d = self.desc
        N = d["grid"]["n_bins"]
        st = np.zeros((len(d["media"]), N), np.float32)
        cdf = np.zeros((max(1, len(d["dyes"])), N), np.float32)
        rho = np.zeros((6, N), np.float32)
        lb = np.zeros(_abi.MAX_LINES, np.int32)
        check(lib().fpt_scene_tables(self._h, st.ctypes.data, cdf.ctypes.data, rho.ctypes.data,
                                     lb.ctypes.data))
        return {"sigma_t": st, "emis_cdf": cdf[: len(d["dyes"])], "rho": rho,
                "line_bin": lb[: len(d["light"]["lines"])]}

    def connection_masks(self):
        """fpt_scene_connection_masks: (geo_clear bits, occluder bits per sphere)."""
        g = C.c_uint32()
        occ = np.zeros(_abi.MAX_SPHERES, np.uint32)
        check(lib().fpt_scene_connection_masks(self._h, C.byref(g), occ.ctypes.data))
        return int(g.value), [int(x) for x in occ[: len(self.desc["geometry"].get("spheres", []))]]

    def new_film(self, batches=1, device="cuda"):
        return torch.zeros(self.film_shape(batches), dtype=torch.float32, device=device)

    def render(self, run: dict, film=None, tallies=None):
        """fpt_render: accumulates into `film` (allocated and zeroed if None)."""
        B = max(1, run.get("parity_batches", 1))
        if film is None:
            film = self.new_film(B)
        _require_cuda(film, torch.float32, "film")
        if film.numel() != int(np.prod(self.film_shape(B))):
            raise ValueError("film has the wrong size")
        if tallies is not None:
            _require_cuda(tallies, torch.int64, "tallies")
        r = _abi.run_struct(run)
        check(lib().fpt_render(self._h, C.byref(r), _ptr(film), _ptr(tallies), _stream()))
        return film

    def render_noalloc(self, run: dict, film, tallies=None):
        """fpt_render_noalloc: fpt_render with the library's static device
        scratch; accumulates into `film` (caller-allocated, like `tallies`)."""
        B = max(1, run.get("parity_batches", 1))
        _require_cuda(film, torch.float32, "film")
        if film.numel() != int(np.prod(self.film_shape(B))):
            raise ValueError("film has the wrong size")
        if tallies is not None:
            _require_cuda(tallies, torch.int64, "tallies")
        r = _abi.run_struct(run)
        check(lib().fpt_render_noalloc(self._h, C.byref(r), _ptr(film), _ptr(tallies), _stream()))
        return film

    def render_adjoint(self, run: dict, grad_film, grad=None, tallies=None):
        """fpt_render_adjoint: accumulates d<grad_film, film>/d theta into `grad`."""
        _require_cuda(grad_film, torch.float32, "grad_film")
        if grad is None:
            grad = torch.zeros(self.n_params, dtype=torch.float32, device=grad_film.device)
        _require_cuda(grad, torch.float32, "grad")
        if tallies is not None:
            _require_cuda(tallies, torch.int64, "tallies")
        r = _abi.run_struct(run)
        check(lib().fpt_render_adjoint(self._h, C.byref(r), _ptr(grad_film), _ptr(grad),
                                       _ptr(tallies), _stream()))
        return grad

    def records(self, run: dict, max_vertices=0, grad_film=None):
        """fpt_render_records: per-path records (numpy structured array on the host)."""
        n = run["path_count"]
        buf = torch.zeros((n, _abi.RECORD_WORDS), dtype=torch.int32, device="cuda")
        rg = None
        if grad_film is not None:
            _require_cuda(grad_film, torch.float32, "grad_film")
            rg = torch.zeros((n, self.n_params), dtype=torch.float32, device="cuda")
        r = _abi.run_struct(run)
        check(lib().fpt_render_records(self._h, C.byref(r), _ptr(buf), max_vertices,
                                       _ptr(grad_film), _ptr(rg), _stream()))
        torch.cuda.synchronize()
        rec = buf.cpu().numpy().view(RECORD_DTYPE).reshape(n)
        return rec, (None if rg is None else rg.cpu().numpy())

    def camera_paths(self, spp):
        """Path count of a camera-side render with spp samples per (pixel, bin)."""
        se = self.desc["sensor"]
        return spp * se["height"] * se["width"] * self.desc["grid"]["n_bins"]

    def render_camera(self, run: dict, film=None, tallies=None):
        """fpt_render_camera: the camera-side estimator; accumulates into
        component 1 of `film` (allocated and zeroed if None).
        run["total_paths"] must be camera_paths(spp)."""
        B = max(1, run.get("parity_batches", 1))
        if film is None:
            film = self.new_film(B)
        _require_cuda(film, torch.float32, "film")
        if film.numel() != int(np.prod(self.film_shape(B))):
            raise ValueError("film has the wrong size")
        if tallies is not None:
            _require_cuda(tallies, torch.int64, "tallies")
        r = _abi.run_struct(run)
        check(lib().fpt_render_camera(self._h, C.byref(r), _ptr(film), _ptr(tallies), None, 0,
                                      _stream()))
        return film

    def camera_records(self, run: dict, max_vertices=0):
        """fpt_render_camera with per-path records only (numpy structured array)."""
        n = run["path_count"]
        buf = torch.zeros((n, _abi.RECORD_WORDS), dtype=torch.int32, device="cuda")
        r = _abi.run_struct(run)
        check(lib().fpt_render_camera(self._h, C.byref(r), None, None, _ptr(buf), max_vertices,
                                      _stream()))
        torch.cuda.synchronize()
        return buf.cpu().numpy().view(RECORD_DTYPE).reshape(n)


RECORD_DTYPE = np.dtype([("n_vertices", "<u4"), ("n_scatter", "<u4"), ("n_emit", "<u4"),
                         ("exit_code", "<u4"), ("lambda", "<i4"), ("comp", "<i4"),
                         ("region", "<i4"), ("pad", "<i4"), ("pos", "<f4", 3),
                         ("dir", "<f4", 3), ("splat_sum", "<f4"), ("pad2", "<f4")])
assert RECORD_DTYPE.itemsize == C.sizeof(_abi.PathRecord)


def new_tallies(n=1, device="cuda"):
    return torch.zeros((n, _abi.N_TALLIES) if n > 1 else (_abi.N_TALLIES,), dtype=torch.int64,
                       device=device)


def tallies_dict(t):
    a = t.detach().cpu().numpy().astype(np.uint64) if isinstance(t, torch.Tensor) else np.asarray(t)
    return {n: int(v) for n, v in zip(TALLY_NAMES, a)}


def render(scene_desc: dict, run: dict):
    """One-shot forward render: returns (film, tallies) on the current device."""
    sc = Scene(scene_desc)
    try:
        t = new_tallies()
        film = sc.render(run, tallies=t)
        return film, t
    finally:
        torch.cuda.synchronize()
        sc.close()


class Batch:
    """Batched form (fpt_batch_create): many escape-sensor slab/sphere instances
    rendered by one persistent launch replayed from a hipGraph."""

    def __init__(self, scenes, runs, tune=None):
        n = len(scenes)
        if n != len(runs) or n == 0:
            raise ValueError("scenes and runs must be non-empty and of equal length")
        self.scenes = scenes
        self.runs = runs
        self.n = n
        self.n_bins = scenes[0]["grid"]["n_bins"]
        descs = [_abi.scene_desc(s) for s in scenes]
        self._descs = (_abi.SceneDesc * n)(*descs)
        self._desc_keep = [d._keep for d in descs]   # tabulated spectra, until created
        self._runs = (_abi.Run * n)(*[_abi.run_struct(r) for r in runs])
        t = None
        if tune is not None:
            t = _abi.Tune(tune.get("block_threads", 0), tune.get("blocks_per_cu", 0),
                          tune.get("refill_lanes", 0), tune.get("chunk_paths", 0),
                          tune.get("block_min_vertices", 0), tune.get("block_segments", 0),
                          tune.get("wide_rounds", 0))
        h = C.c_void_p()
        check(lib().fpt_batch_create(self._descs, self._runs, n, None if t is None else C.byref(t),
                                     C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().fpt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def new_films(self, device="cuda"):
        return torch.zeros((self.n, 2, 2, self.n_bins), dtype=torch.float32, device=device)

    def render(self, films, tallies=None):
        _require_cuda(films, torch.float32, "films")
        if films.numel() != self.n * 4 * self.n_bins:
            raise ValueError("films has the wrong size")
        if tallies is not None:
            _require_cuda(tallies, torch.int64, "tallies")
            if tallies.numel() != self.n * _abi.N_TALLIES:
                raise ValueError("tallies has the wrong size")
        check(lib().fpt_batch_render(self._h, _ptr(films), _ptr(tallies), _stream()))
        return films

    def count_vertices(self):
        films = self.new_films()
        t = new_tallies(self.n)
        self.render(films, t)
        torch.cuda.synchronize()
        return int(t[:, 1].sum().item())
