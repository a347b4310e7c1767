"""Python binding of libgal.so (the C ABI in include/gal.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the ABI.  PyTorch provides device memory (tensors) and the
stream.  If the library has not been built, loading fails loudly; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgal.so")

GAL_OK = 0
GAL_COLOR = 0x1
GAL_MANIP = 0x2
GAL_SLIDE = 0x4
GAL_LINKS = 0x8
GAL_SHADE = 0x10
ERRORS = {-1: "GAL_EINVAL", -2: "GAL_ENOMEM", -3: "GAL_EDEVICE", -4: "GAL_ESTATE",
          -5: "GAL_EOVERFLOW"}

_fp = C.POINTER(C.c_float)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u8p = C.POINTER(C.c_uint8)
_u32p = C.POINTER(C.c_uint32)


class GalRobot(C.Structure):
    _fields_ = [("dh", C.c_float * 28), ("qlim", C.c_float * 14), ("q_home", C.c_float * 7),
                ("mount", C.c_float * 3), ("cam_offset", C.c_float * 3),
                ("cam_pitch_cs", C.c_float * 2), ("num_spheres", C.c_int32),
                ("sphere_link", _i32p), ("sphere_pos", _fp), ("sphere_class", _i32p),
                ("sphere_held_only", _u8p), ("grasp_tip", C.c_float * 3),
                ("grasp_radius", C.c_float), ("held_class", C.c_int32),
                ("link_box", _fp), ("link_rgb", _u8p)]


class GalSceneSet(C.Structure):
    _fields_ = [("num_envs", C.c_int32), ("vert_offset", _i64p), ("verts", _fp),
                ("tri_offset", _i64p), ("tris", _i32p), ("tri_rgb", _u8p),
                ("box_offset", _i64p), ("boxes", _fp), ("num_objects", C.c_int32),
                ("objects", _fp), ("grid_origin", _fp), ("grid_dims", _i32p),
                ("num_starts", C.c_int32), ("starts", _fp), ("held", _u8p), ("res", _i32p),
                ("tri_plane", _fp), ("obj_rgb", _u8p)]


class GalConfig(C.Structure):
    _fields_ = [("res0", C.c_int32), ("near_m", C.c_float), ("far_m", C.c_float),
                ("cell_m", C.c_float), ("num_classes", C.c_int32),
                ("class_radius", C.c_float * 8), ("act_lim", C.c_float * 3),
                ("episode_len", C.c_int32), ("flags", C.c_uint32),
                ("slide_step", C.c_float), ("place_step", C.c_float), ("manip_seed", C.c_uint64)]


class GalTuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("region", C.c_int32), ("lane_max", C.c_int32),
                ("small_max", C.c_int32),
                ("refresh", C.c_int32), ("occlusion", C.c_int32), ("prologue", C.c_int32),
                ("persistent", C.c_int32), ("robot_lanes", C.c_int32), ("graph", C.c_int32),
                ("split", C.c_int32), ("order", C.c_int32), ("objgrid", C.c_int32),
                ("bin", C.c_int32), ("layer_cache", C.c_int32)]


class GalOutputs(C.Structure):
    _fields_ = [("depth", C.c_void_p), ("rgb", C.c_void_p), ("contact_static", C.c_void_p),
                ("contact_object", C.c_void_p), ("accepted", C.c_void_p), ("state", C.c_void_p),
                ("frames", C.c_void_p), ("counters", C.c_void_p), ("done", C.c_void_p),
                ("object_frames", C.c_void_p), ("held", C.c_void_p)]


_lib = None


def load_library():
    """Load libgal.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2306_07552_amd.build` "
                "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        L.gal_create_batch.argtypes = [C.POINTER(GalConfig), C.POINTER(GalRobot),
                                       C.POINTER(GalSceneSet), C.c_void_p, C.POINTER(C.c_void_p)]
        L.gal_reset.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.gal_step.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(GalOutputs), C.c_void_p]
        L.gal_batch_info.argtypes = [C.c_void_p, _i32p, _i32p, _i32p, _i64p]
        L.gal_depth_offsets.argtypes = [C.c_void_p, _i64p, C.c_size_t]
        L.gal_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.gal_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.gal_get_grid.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _u32p, C.c_size_t, _fp,
                                   C.c_size_t, _i64p]
        L.gal_profile_enable.argtypes = [C.c_void_p, C.c_int]
        L.gal_profile_read.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       _i64p]
        L.gal_profile_read_stages.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_size_t, _i64p]
        L.gal_mesh_info.argtypes = [C.c_void_p, _i64p, _i64p, _i64p]
        L.gal_counters_enable.argtypes = [C.c_void_p, C.c_int]
        L.gal_counters_read.argtypes = [C.c_void_p, _i64p, C.c_size_t]
        L.gal_autotune.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(GalOutputs), C.c_void_p,
                                   C.c_int32, C.POINTER(GalTuning), C.POINTER(C.c_double)]
        L.gal_get_tuning.argtypes = [C.c_void_p, C.POINTER(GalTuning)]
        L.gal_mlp_num_params.argtypes = [_i64p]
        L.gal_mlp_create.argtypes = [C.c_int32, C.c_uint64, C.POINTER(C.c_void_p)]
        L.gal_mlp_set_weights.argtypes = [C.c_void_p, _fp, C.c_size_t]
        L.gal_mlp_get_weights.argtypes = [C.c_void_p, _fp, C.c_size_t]
        L.gal_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.gal_mlp_forward_static.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                             C.c_void_p]
        L.gal_mlp_gradients.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                        C.c_void_p, C.c_void_p, C.c_void_p]
        L.gal_mlp_train_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                         C.c_float, C.c_void_p, C.c_void_p]
        L.gal_mlp_gemm_test.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                        C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                        C.c_void_p]
        L.gal_mlp_destroy.argtypes = [C.c_void_p]
        L.gal_mlp_destroy.restype = None
        L.gal_policy_create.argtypes = [C.c_int32, C.c_int32, C.c_uint64, C.POINTER(C.c_void_p)]
        L.gal_policy_num_params.argtypes = [C.c_void_p, _i64p]
        L.gal_policy_set_weights.argtypes = [C.c_void_p, _fp, C.c_size_t]
        L.gal_policy_get_weights.argtypes = [C.c_void_p, _fp, C.c_size_t]
        L.gal_policy_act.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.gal_policy_activations.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_uint16), C.c_size_t]
        L.gal_policy_ppo_gradients.argtypes = [C.c_void_p] + [C.c_void_p] * 6 + [C.c_int32, C.c_void_p,
                                                                                  C.c_void_p, C.c_void_p, C.c_void_p]
        L.gal_policy_adam_step.argtypes = [C.c_void_p, C.c_float, C.c_void_p]
        L.gal_gae.argtypes = [C.c_void_p] * 4 + [C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_void_p,
                                                 C.c_void_p, C.c_void_p]
        L.gal_policy_destroy.argtypes = [C.c_void_p]
        L.gal_policy_destroy.restype = None
        L.gal_features.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.gal_surrogate_attach.argtypes = [C.c_void_p, C.c_void_p, C.c_float, C.c_uint32, C.c_void_p]
        L.gal_surrogate_logits.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.gal_surrogate_detach.argtypes = [C.c_void_p]
        L.gal_surrogate_stats.argtypes = [C.c_void_p, _i64p, C.c_int]
        L.gal_set_tuning.argtypes = [C.c_void_p, C.POINTER(GalTuning)]
        L.gal_destroy.argtypes = [C.c_void_p]
        L.gal_destroy.restype = None
        L.gal_last_error.restype = C.c_char_p
        _lib = L
    return _lib


class GalError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(rc: int):
    if rc != GAL_OK:
        raise GalError(rc, load_library().gal_last_error().decode())


def _p(a: Optional[np.ndarray], t):
    if a is None:
        return C.cast(None, t)
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(t)


def _need(a, shape, name):
    if tuple(np.shape(a)) != tuple(shape):
        raise GalError(-1, f"{name}: shape {tuple(np.shape(a))}, expected {tuple(shape)}")


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Batch:
    """A batch of environments stepped together on one GPU."""

    def __init__(self, robot, scenes, consts: dict, color: bool = False, stream=None):
        L = load_library()
        keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dt)
            keep.append(a)
            return a

        cfg = GalConfig()
        cfg.res0 = int(consts["res0"])
        cfg.near_m = float(np.float32(consts["near"]))
        cfg.far_m = float(np.float32(consts["far"]))
        cfg.cell_m = float(np.float32(consts["cell"]))
        rc = list(consts["radius_classes"])
        cfg.num_classes = len(rc)
        cfg.class_radius[:] = [float(np.float32(v)) for v in rc] + [0.0] * (8 - len(rc))
        cfg.act_lim[:] = [float(np.float32(v)) for v in consts["act_lim"]]
        cfg.episode_len = int(consts["episode_len"])
        cfg.flags = GAL_COLOR if color else 0
        self.manip = bool(consts.get("manip", False))
        if self.manip:
            cfg.flags |= GAL_MANIP | (GAL_SLIDE if consts.get("slide", False) else 0)
            cfg.slide_step = float(np.float32(consts["slide_step"]))
            cfg.place_step = float(np.float32(consts["place_step"]))
            cfg.manip_seed = int(consts["seed"])

        r = GalRobot()
        r.dh[:] = [float(v) for v in np.asarray(robot.dh, np.float32).ravel()]
        r.qlim[:] = [float(v) for v in np.asarray(robot.qlim, np.float32).ravel()]
        r.q_home[:] = [float(v) for v in np.asarray(robot.q_home, np.float32)]
        r.mount[:] = [float(v) for v in np.asarray(robot.mount, np.float32)]
        r.cam_offset[:] = [float(v) for v in np.asarray(robot.cam_offset, np.float32)]
        r.cam_pitch_cs[:] = [float(v) for v in np.asarray(robot.cam_pitch_cs, np.float32)]
        r.num_spheres = int(robot.num_spheres)
        r.sphere_link = _p(arr(robot.sphere_link, np.int32), _i32p)
        r.sphere_pos = _p(arr(robot.sphere_pos, np.float32), _fp)
        r.sphere_class = _p(arr(robot.sphere_class, np.int32), _i32p)
        r.sphere_held_only = _p(arr(robot.sphere_held_only, np.uint8), _u8p)
        if color and consts.get("shade", False):
            cfg.flags |= GAL_SHADE
        self.links = bool(consts.get("links", False))
        if self.links:
            cfg.flags |= GAL_LINKS
            _need(robot.link_box, (8, 6), "link_box")
            r.link_box = _p(arr(robot.link_box, np.float32), _fp)
            if robot.link_rgb is not None:
                _need(robot.link_rgb, (8, 3), "link_rgb")
                r.link_rgb = _p(arr(robot.link_rgb, np.uint8), _u8p)
        if self.manip:
            r.grasp_tip[:] = [float(v) for v in np.asarray(consts["grasp_tip"], np.float32)]
            r.grasp_radius = float(np.float32(consts["grasp_radius"]))
            r.held_class = int(consts["held_class"])

        s = GalSceneSet()
        S = scenes
        # the C ABI takes the arrays without lengths: their shapes must agree
        # with the offsets before the library reads them
        N = int(S.num_envs)
        T = int(np.asarray(S.tri_offset)[-1])
        _need(S.vert_offset, (N + 1,), "vert_offset")
        _need(S.tri_offset, (N + 1,), "tri_offset")
        _need(S.box_offset, (N + 1,), "box_offset")
        _need(S.verts, (int(np.asarray(S.vert_offset)[-1]), 3), "verts")
        _need(S.tris, (T, 3), "tris")
        _need(S.tri_rgb, (T, 3), "tri_rgb")
        _need(S.boxes, (int(np.asarray(S.box_offset)[-1]), 6), "boxes")
        _need(S.objects, (N, int(S.num_objects), 8), "objects")
        _need(S.grid_origin, (N, 2), "grid_origin")
        _need(S.grid_dims, (N, 2), "grid_dims")
        _need(S.starts, (N, int(S.num_starts), 3), "starts")
        _need(S.held, (N,), "held")
        _need(S.res, (N,), "res")
        if getattr(S, "tri_plane", None) is not None:
            _need(S.tri_plane, (T, 4), "tri_plane")
        s.num_envs = int(S.num_envs)
        s.vert_offset = _p(arr(S.vert_offset, np.int64), _i64p)
        s.verts = _p(arr(S.verts, np.float32), _fp)
        s.tri_offset = _p(arr(S.tri_offset, np.int64), _i64p)
        s.tris = _p(arr(S.tris, np.int32), _i32p)
        s.tri_rgb = _p(arr(S.tri_rgb, np.uint8), _u8p)
        s.box_offset = _p(arr(S.box_offset, np.int64), _i64p)
        s.boxes = _p(arr(S.boxes, np.float32), _fp)
        s.num_objects = int(S.num_objects)
        s.objects = _p(arr(S.objects, np.float32), _fp)
        s.grid_origin = _p(arr(S.grid_origin, np.float32), _fp)
        s.grid_dims = _p(arr(S.grid_dims, np.int32), _i32p)
        s.num_starts = int(S.num_starts)
        s.starts = _p(arr(S.starts, np.float32), _fp)
        s.held = _p(arr(S.held, np.uint8), _u8p)
        s.res = _p(arr(S.res, np.int32), _i32p)
        tp = getattr(S, "tri_plane", None)
        s.tri_plane = _p(arr(tp, np.float32), _fp) if tp is not None else None
        orgb = getattr(S, "obj_rgb", None)
        if orgb is not None:
            _need(orgb, (N, int(S.num_objects), 3), "obj_rgb")
        s.obj_rgb = _p(arr(orgb, np.uint8), _u8p) if orgb is not None else None
        self.num_objects = int(S.num_objects)

        h = C.c_void_p()
        _check(L.gal_create_batch(C.byref(cfg), C.byref(r), C.byref(s),
                                  _stream_handle(stream), C.byref(h)))
        self._h = h
        self.color = color
        n, sp, w, px = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        _check(L.gal_batch_info(h, C.byref(n), C.byref(sp), C.byref(w), C.byref(px)))
        self.num_envs, self.num_spheres, self.contact_words = n.value, sp.value, w.value
        self.depth_pixels = px.value
        off = np.zeros(self.num_envs + 1, np.int64)
        _check(L.gal_depth_offsets(h, _p(off, _i64p), off.size))
        self.depth_off = off
        self.res = np.asarray(S.res, np.int32).copy()

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gal_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc_outputs(self, device="cuda") -> Dict[str, "object"]:
        import torch
        N, W = self.num_envs, self.contact_words
        out = dict(
            depth=torch.empty(self.depth_pixels, dtype=torch.int32, device=device),
            contact_static=torch.empty((N, W), dtype=torch.int32, device=device),
            contact_object=torch.empty((N, W), dtype=torch.int32, device=device),
            accepted=torch.empty(N, dtype=torch.uint8, device=device),
            state=torch.empty((N, 10), dtype=torch.float32, device=device),
            frames=torch.empty((N, 8, 12), dtype=torch.float32, device=device),
            counters=torch.empty((N, 2), dtype=torch.int32, device=device),
            done=torch.empty(N, dtype=torch.uint8, device=device),
        )
        if self.color:
            out["rgb"] = torch.empty((self.depth_pixels, 3), dtype=torch.uint8, device=device)
        if self.manip:
            out["object_frames"] = torch.empty((N, self.num_objects, 12), dtype=torch.float32,
                                               device=device)
            out["held"] = torch.empty(N, dtype=torch.int32, device=device)
        return out

    @staticmethod
    def _outputs(out) -> GalOutputs:
        o = GalOutputs()
        for k in ("depth", "rgb", "contact_static", "contact_object", "accepted", "state",
                  "frames", "counters", "done", "object_frames", "held"):
            setattr(o, k, _ptr(out.get(k)))
        return o

    def step(self, actions, out: Dict[str, "object"], stream=None):
        o = self._outputs(out)
        assert actions.is_contiguous() and actions.dtype.is_floating_point
        _check(load_library().gal_step(self._h, actions.data_ptr(), C.byref(o),
                                       _stream_handle(stream)))

    def autotune(self, actions, out: Dict[str, "object"], steps: int = 5, stream=None):
        """Pick the fastest launch configuration (same bits for all); returns
        (tuning dict, ms per step)."""
        o = self._outputs(out)
        t = GalTuning()
        ms = C.c_double()
        _check(load_library().gal_autotune(self._h, actions.data_ptr(), C.byref(o),
                                           _stream_handle(stream), steps, C.byref(t), C.byref(ms)))
        return {k: getattr(t, k) for k, _ in GalTuning._fields_}, ms.value

    def reset(self, mask=None, stream=None):
        _check(load_library().gal_reset(self._h, _ptr(mask), _stream_handle(stream)))

    def _state_words(self):
        N, O = self.num_envs, self.num_objects
        return N * 12 + (N * (8 * O + 1 + 12) if self.manip else 0)

    def get_state(self, stream=None, manip: bool = False):
        """(state [N][10], counters [N][2]); with manip=True (GAL_MANIP batches)
        also objects [N][O][8], held [N], rel [N][12]."""
        N, O = self.num_envs, self.num_objects
        buf = np.zeros(self._state_words(), np.float32)
        _check(load_library().gal_get_state(self._h, buf.ctypes.data, buf.nbytes,
                                            _stream_handle(stream)))
        st = buf[:N * 10].reshape(N, 10).copy()
        cnt = buf[N * 10:N * 12].view(np.int32).reshape(N, 2).copy()
        if not manip:
            return st, cnt
        k = N * 12
        objs = buf[k:k + N * O * 8].reshape(N, O, 8).copy()
        k += N * O * 8
        held = buf[k:k + N].view(np.int32).copy()
        k += N
        rel = buf[k:k + N * 12].reshape(N, 12).copy()
        return st, cnt, objs, held, rel

    def set_state(self, state: np.ndarray, counters: np.ndarray, objects=None, held=None, rel=None,
                  stream=None):
        N = self.num_envs
        parts = [np.ascontiguousarray(state, np.float32).ravel(),
                 np.ascontiguousarray(counters, np.int32).ravel().view(np.float32)]
        if self.manip:
            if objects is None:
                _, _, objects, held, rel = self.get_state(stream, manip=True)
            parts += [np.ascontiguousarray(objects, np.float32).ravel(),
                      np.ascontiguousarray(held, np.int32).ravel().view(np.float32),
                      np.ascontiguousarray(rel, np.float32).ravel()]
        buf = np.concatenate(parts)
        assert buf.size == self._state_words()
        _check(load_library().gal_set_state(self._h, buf.ctypes.data, buf.nbytes,
                                            _stream_handle(stream)))

    def get_grid(self, env: int, cls: int, nx: int, ny: int):
        L = load_library()
        n = C.c_int64()
        _check(L.gal_get_grid(self._h, env, cls, C.cast(None, _u32p), 0, C.cast(None, _fp), 0,
                              C.byref(n)))
        offs = np.zeros(nx * ny + 1, np.uint32)
        lay = np.zeros((max(n.value, 1), 2), np.float32)
        _check(L.gal_get_grid(self._h, env, cls, _p(offs, _u32p), offs.size, _p(lay, _fp),
                              n.value, C.byref(n)))
        return offs, lay[:n.value]

    # ---- collision surrogate
    def features(self, actions, x, stream=None):
        """BF16 surrogate inputs (torch int16 [N][2112]) of the next move."""
        _check(load_library().gal_features(self._h, actions.data_ptr(), x.data_ptr(),
                                           _stream_handle(stream)))

    def attach_surrogate(self, mlp: "Mlp", skip_below: float, audit_period: int = 16,
                         stream=None):
        _check(load_library().gal_surrogate_attach(self._h, mlp._h, float(skip_below),
                                                   int(audit_period), _stream_handle(stream)))
        self._mlp = mlp   # keep it alive while attached

    def surrogate_logits(self, actions, logits, stream=None):
        """Logits (torch float32 [N]) of the attached surrogate for the next move."""
        _check(load_library().gal_surrogate_logits(self._h, actions.data_ptr(), logits.data_ptr(),
                                                   _stream_handle(stream)))

    def detach_surrogate(self):
        _check(load_library().gal_surrogate_detach(self._h))
        self._mlp = None

    def surrogate_stats(self, reset: bool = False) -> dict:
        v = np.zeros(4, np.int64)
        _check(load_library().gal_surrogate_stats(self._h, _p(v, _i64p), 1 if reset else 0))
        return dict(queries=int(v[0]), skipped=int(v[1]), audited=int(v[2]),
                    mismatches=int(v[3]))

    def get_tuning(self) -> dict:
        t = GalTuning()
        _check(load_library().gal_get_tuning(self._h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in GalTuning._fields_}

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = GalTuning(**cur)
        _check(load_library().gal_set_tuning(self._h, C.byref(t)))

    COUNTERS = ("clusters_tested", "clusters_in_frustum", "clusters_occluded", "clusters_drawn",
                "tris_valid", "tris_clipped", "tris_setup", "cand_pixels")

    def counters(self, on: bool):
        _check(load_library().gal_counters_enable(self._h, 1 if on else 0))

    def counters_read(self) -> dict:
        v = np.zeros(len(self.COUNTERS), np.int64)
        _check(load_library().gal_counters_read(self._h, _p(v, _i64p), v.size))
        return dict(zip(self.COUNTERS, (int(x) for x in v)))

    def profile(self, on: bool):
        _check(load_library().gal_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """(robot-step ms, raster ms, steps) summed over the recorded steps."""
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        _check(load_library().gal_profile_read(self._h, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value

    def profile_read_stages(self):
        """(surrogate ms, robot-step ms, raster ms, steps) summed over the recorded steps."""
        v = (C.c_double * 3)()
        n = C.c_int64()
        _check(load_library().gal_profile_read_stages(self._h, v, 3, C.byref(n)))
        return v[0], v[1], v[2], n.value

    def mesh_info(self):
        c, v, t = C.c_int64(), C.c_int64(), C.c_int64()
        _check(load_library().gal_mesh_info(self._h, C.byref(c), C.byref(v), C.byref(t)))
        return dict(clusters=c.value, cluster_verts=v.value, tris=t.value)

    def env_depth(self, depth_flat, e: int):
        r = int(self.res[e])
        return depth_flat[int(self.depth_off[e]):int(self.depth_off[e + 1])].reshape(r, r)


class Mlp:
    """The collision-surrogate MLP on the device (see include/gal.h)."""
    IN = 2112

    def __init__(self, max_rows: int, seed: int = 0):
        L = load_library()
        h = C.c_void_p()
        _check(L.gal_mlp_create(int(max_rows), int(seed), C.byref(h)))
        self._h = h
        self.max_rows = int(max_rows)
        n = C.c_int64()
        _check(L.gal_mlp_num_params(C.byref(n)))
        self.num_params = n.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gal_mlp_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_weights(self) -> np.ndarray:
        w = np.zeros(self.num_params, np.float32)
        _check(load_library().gal_mlp_get_weights(self._h, _p(w, _fp), w.size))
        return w

    def set_weights(self, w: np.ndarray):
        w = np.ascontiguousarray(w, np.float32)
        _check(load_library().gal_mlp_set_weights(self._h, _p(w, _fp), w.size))

    def forward(self, x, logits, rows=None, stream=None):
        rows = x.shape[0] if rows is None else rows
        _check(load_library().gal_mlp_forward(self._h, x.data_ptr(), int(rows), logits.data_ptr(),
                                              _stream_handle(stream)))

    def forward_static(self, x, logits, rows=None, stream=None):
        """gal_mlp_forward_static: the same logits, scratch in the library's fixed array."""
        rows = x.shape[0] if rows is None else rows
        _check(load_library().gal_mlp_forward_static(self._h, x.data_ptr(), int(rows),
                                                     logits.data_ptr(), _stream_handle(stream)))

    def gradients(self, x, y, pos_weight, grads=None, loss=None, stream=None):
        _check(load_library().gal_mlp_gradients(self._h, x.data_ptr(), y.data_ptr(), x.shape[0],
                                                float(pos_weight), _ptr(grads), _ptr(loss),
                                                _stream_handle(stream)))

    def train_step(self, x, y, pos_weight, lr, loss=None, stream=None):
        _check(load_library().gal_mlp_train_step(self._h, x.data_ptr(), y.data_ptr(), x.shape[0],
                                                 float(pos_weight), float(lr), _ptr(loss),
                                                 _stream_handle(stream)))

    @staticmethod
    def layout():
        """(offset, shape) of W1, b1, ..., W5, b5 in the flat parameter vector."""
        dims = [2112, 256, 256, 256, 256, 1]
        out, off = [], 0
        for l in range(5):
            n = dims[l + 1] * dims[l]
            out.append((off, (dims[l + 1], dims[l])))
            off += n
            out.append((off, (dims[l + 1],)))
            off += dims[l + 1]
        return out


def gemm_test(variant, a, b, M, N, K, lda, ldb, c, ldc, stream=None):
    _check(load_library().gal_mlp_gemm_test(variant, a.data_ptr(), b.data_ptr(), M, N, K, lda, ldb,
                                            c.data_ptr(), ldc, _stream_handle(stream)))


class Policy:
    """The policy network that consumes the depth stack (see include/gal.h)."""

    def __init__(self, max_envs: int, act_dim: int = 9, seed: int = 0):
        L = load_library()
        h = C.c_void_p()
        _check(L.gal_policy_create(int(max_envs), int(act_dim), int(seed), C.byref(h)))
        self._h = h
        self.max_envs = int(max_envs)
        self.act_dim = int(act_dim)
        n = C.c_int64()
        _check(L.gal_policy_num_params(h, C.byref(n)))
        self.num_params = n.value
        self._last = 0

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gal_policy_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_weights(self) -> np.ndarray:
        w = np.zeros(self.num_params, np.float32)
        _check(load_library().gal_policy_get_weights(self._h, _p(w, _fp), w.size))
        return w

    def set_weights(self, w: np.ndarray):
        w = np.ascontiguousarray(w, np.float32)
        _check(load_library().gal_policy_set_weights(self._h, _p(w, _fp), w.size))

    def act(self, depth, state, actions, noise=None, value=None, logp=None, n_envs=None, stream=None):
        """depth: the batch's depth output (128x128 images, read in place)."""
        n = int(state.shape[0]) if n_envs is None else int(n_envs)
        _check(load_library().gal_policy_act(self._h, depth.data_ptr(), state.data_ptr(), n, _ptr(noise),
                                             actions.data_ptr(), _ptr(value), _ptr(logp),
                                             _stream_handle(stream)))
        self._last = n

    def ppo_gradients(self, depth, state, actions, old_logp, adv, ret, clip=0.2, value_coef=0.5,
                      entropy_coef=0.01, grads=None, stats=None, samples=None, stream=None):
        """One PPO gradient over the samples (kept for adam_step; copied to
        `grads` when given); `stats` (4 floats): policy loss, value error,
        entropy, mean ratio."""
        S = int(state.shape[0]) if samples is None else int(samples)
        hp = GalPpoParams(float(clip), float(value_coef), float(entropy_coef))
        _check(load_library().gal_policy_ppo_gradients(self._h, depth.data_ptr(), state.data_ptr(),
                                                       actions.data_ptr(), old_logp.data_ptr(), adv.data_ptr(),
                                                       ret.data_ptr(), S, C.cast(C.pointer(hp), C.c_void_p),
                                                       _ptr(grads), _ptr(stats), _stream_handle(stream)))
        self._last = S

    def adam_step(self, lr, stream=None):
        _check(load_library().gal_policy_adam_step(self._h, float(lr), _stream_handle(stream)))

    SHAPES = {1: (31, 31, 32), 2: (14, 14, 64), 3: (12, 12, 32), 4: (512,)}

    def activations(self, layer: int) -> np.ndarray:
        """Layer 1..4 activations of the last act (BF16 bit patterns)."""
        shp = (self._last,) + self.SHAPES[layer]
        out = np.zeros(shp, np.uint16)
        _check(load_library().gal_policy_activations(self._h, int(layer),
                                                     out.ctypes.data_as(C.POINTER(C.c_uint16)), out.size))
        return out


class GalPpoParams(C.Structure):
    _fields_ = [("clip", C.c_float), ("value_coef", C.c_float), ("entropy_coef", C.c_float)]


def gae(rewards, values, dones, last_value, gamma, lam, adv, ret, stream=None):
    """Generalised advantage estimation over a rollout [T][N] on the device."""
    T, N = int(rewards.shape[0]), int(rewards.shape[1])
    _check(load_library().gal_gae(rewards.data_ptr(), values.data_ptr(), dones.data_ptr(), last_value.data_ptr(),
                                  T, N, float(gamma), float(lam), adv.data_ptr(), ret.data_ptr(),
                                  _stream_handle(stream)))
