"""ctypes loader for libhpvm_sgemm.so.

torch is imported first so that its HIP runtime (soname libamdhip64.so.7) is
the one the library binds to; torch's device pointers and streams are then
valid inside the library.  There is no fallback: if the library is missing
the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libhpvm_sgemm.so")

i32 = ctypes.c_int32
i64 = ctypes.c_int64
f32 = ctypes.c_float
vp = ctypes.c_void_p


class Tile(ctypes.Structure):
    _fields_ = [("tile_m", i32), ("tile_n", i32), ("tile_k", i32),
                ("leaf_m", i32), ("leaf_n", i32), ("stages", i32)]

    def as_tuple(self):
        return (self.tile_m, self.tile_n, self.tile_k, self.leaf_m, self.leaf_n, self.stages)


class RootIn(ctypes.Structure):
    _pack_ = 1
    _fields_ = [("A", vp), ("bytesA", i64), ("lda", i32),
                ("B", vp), ("bytesB", i64), ("ldb", i32),
                ("C", vp), ("bytesC", i64), ("ldc", i32),
                ("k", i32), ("alpha", f32), ("beta", f32),
                ("block_x", i32), ("block_y", i32), ("grid_x", i32), ("grid_y", i32)]


class Dfg(ctypes.Structure):
    _fields_ = [("root_instances", i32), ("grid_x", i32), ("grid_y", i32),
                ("block_x", i32), ("block_y", i32), ("waves", i32),
                ("alloc_bytes", i64), ("k_slabs", i32), ("lowering", i32),
                ("splits", i32), ("reserved", i32), ("tile", Tile)]


class Edge(ctypes.Structure):
    _fields_ = [("kind", i32), ("src_node", i32), ("dst_node", i32),
                ("src_port", i32), ("dst_port", i32), ("all_to_all", i32)]


class SgemmDesc(ctypes.Structure):
    _fields_ = [("m", i64), ("n", i64), ("k", i64), ("alpha", f32), ("beta", f32),
                ("A", vp), ("lda", i64), ("B", vp), ("ldb", i64), ("C", vp), ("ldc", i64)]


class Consumer(ctypes.Structure):
    _fields_ = [("op", i32), ("reserved", i32), ("bias", vp), ("lo", f32), ("hi", f32)]


class Tracked(ctypes.Structure):
    _fields_ = [("start", vp), ("bytes", i64), ("device", vp), ("on_host", i32), ("on_device", i32)]


class TrackerStats(ctypes.Structure):
    _fields_ = [("h2d_bytes", i64), ("h2d_copies", i64), ("d2h_bytes", i64), ("d2h_copies", i64),
                ("launches", i64), ("regions", i64)]


class StreamConfig(ctypes.Structure):
    _fields_ = [("capacity", i32), ("grid", i32), ("idle_ms", i32), ("reserved", i32)]


class StreamStatus(ctypes.Structure):
    _fields_ = [("pushed", i64), ("popped", i64), ("tiles", i64), ("capacity", i32), ("grid", i32),
                ("idle_ms", i32), ("running", i32), ("idle_ended", i32), ("reserved", i32)]


class GroupedInfo(ctypes.Structure):
    _fields_ = [("count", i32), ("total_tiles", i32), ("grid", i32), ("shapes_used", i32),
                ("workspace_bytes", i64), ("scratch_bytes", i64), ("flops", ctypes.c_double)]


PTile = ctypes.POINTER(Tile)
Pvp = ctypes.POINTER(vp)
Pi64 = ctypes.POINTER(i64)

# name -> (restype, argtypes); the same list the header declares.
SIGNATURES = {
    "hpvm_sgemm": (ctypes.c_int, [i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, i32,
                                  ctypes.POINTER(Tile), vp]),
    "hpvm_launch_root": (ctypes.c_int, [ctypes.POINTER(RootIn), vp]),
    "hpvm_wait": (ctypes.c_int, [vp]),
    "hpvm_alloc_bytes": (ctypes.c_int, [ctypes.POINTER(Tile), i32, ctypes.POINTER(i64)]),
    "hpvm_describe": (ctypes.c_int, [i64, i64, i64, i32, ctypes.POINTER(Tile), ctypes.POINTER(Dfg)]),
    "hpvm_describe_ws": (ctypes.c_int, [i64, i64, i64, i32, ctypes.POINTER(Tile), i64, ctypes.POINTER(Dfg)]),
    "hpvm_dfg_edges": (ctypes.c_int, [ctypes.POINTER(Edge), i32, ctypes.POINTER(i32)]),
    "hpvm_tile_menu": (ctypes.c_int, [i32, ctypes.POINTER(Tile), i32, ctypes.POINTER(i32)]),
    "hpvm_grouped_plan_create": (ctypes.c_int, [i32, ctypes.POINTER(SgemmDesc), i32, PTile, Pvp]),
    "hpvm_grouped_plan_info": (ctypes.c_int, [vp, ctypes.POINTER(GroupedInfo)]),
    "hpvm_grouped_instance_tile": (ctypes.c_int, [vp, i32, PTile]),
    "hpvm_grouped_menu": (ctypes.c_int, [PTile, i32, ctypes.POINTER(i32)]),
    "hpvm_grouped_workspace_bytes": (ctypes.c_int, [vp, Pi64]),
    "hpvm_grouped_run": (ctypes.c_int, [vp, vp, i64, vp]),
    "hpvm_grouped_capture": (ctypes.c_int, [vp, vp, i64, vp, Pvp]),
    "hpvm_graph_launch": (ctypes.c_int, [vp, vp]),
    "hpvm_graph_destroy": (ctypes.c_int, [vp]),
    "hpvm_grouped_plan_destroy": (ctypes.c_int, [vp]),
    "hpvm_grouped_autotune": (ctypes.c_int, [vp, vp, i64, vp, i64, i32, vp, ctypes.POINTER(f32)]),
    "hpvm_autotune": (ctypes.c_int, [i64, i64, i64, i32, vp, i64, vp, i64, vp, i64, vp, i64, i32, vp,
                                     PTile, ctypes.POINTER(f32)]),
    "hpvm_sgemm_ws": (ctypes.c_int, [i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, i32, PTile, vp, i64,
                                     vp]),
    "hpvm_sgemm_workspace_bytes": (ctypes.c_int, [i64, i64, i64, i32, PTile, Pi64]),
    "hpvm_sgemm_noalloc": (ctypes.c_int, [i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, i32, PTile,
                                          vp]),
    "hpvm_autotune_lookup": (ctypes.c_int, [i64, i64, i64, i32, PTile, ctypes.POINTER(i32)]),
    "hpvm_autotune_record": (ctypes.c_int, [i64, i64, i64, i32, PTile, f32]),
    "hpvm_autotune_clear": (ctypes.c_int, []),
    "hpvm_autotune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "hpvm_autotune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "hpvm_sgemm_backward_workspace_bytes": (ctypes.c_int, [i64, i64, i64, i32, PTile, Pi64]),
    "hpvm_sgemm_backward": (ctypes.c_int, [i64, i64, i64, f32, f32, vp, i64, vp, i64, vp, i64, vp, i64,
                                           vp, i64, vp, i64, vp, i64, vp, vp, i32, PTile, vp, i64, vp]),
    "hpvm_sgemm_backward_menu": (ctypes.c_int, [i32, PTile, i32, ctypes.POINTER(i32)]),
    "hpvm_autotune_backward": (ctypes.c_int, [i64, i64, i64, i32, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64,
                                              vp, i64, i32, vp, PTile, ctypes.POINTER(f32)]),
    "hpvm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "hpvm_last_error": (ctypes.c_char_p, []),
    "hpvm_fusion_menu": (ctypes.c_int, [i32, ctypes.POINTER(Tile), i32, ctypes.POINTER(i32)]),
    "hpvm_sgemm_consumer": (ctypes.c_int, [i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64,
                                           ctypes.POINTER(Consumer), vp, i64, ctypes.POINTER(Tile), vp]),
    "hpvm_sgemm_pair": (ctypes.c_int, [i64, i64, i64, vp, i64, f32, vp, i64, f32, vp, i64,
                                       f32, vp, i64, f32, vp, i64, ctypes.POINTER(Tile), vp]),
    "hpvm_sgemm_pair_ws": (ctypes.c_int, [i64, i64, i64, vp, i64, f32, vp, i64, f32, vp, i64,
                                          f32, vp, i64, f32, vp, i64, ctypes.POINTER(Tile), vp, i64, vp]),
    "hpvm_sgemm_pair_workspace_bytes": (ctypes.c_int, [i64, i64, i64, ctypes.POINTER(Tile), Pi64]),
    "hpvm_track_mem": (ctypes.c_int, [vp, i64]),
    "hpvm_request_mem": (ctypes.c_int, [vp, i64, vp]),
    "hpvm_untrack_mem": (ctypes.c_int, [vp, vp]),
    "hpvm_tracked_state": (ctypes.c_int, [vp, ctypes.POINTER(Tracked)]),
    "hpvm_tracker_counters": (ctypes.c_int, [ctypes.POINTER(TrackerStats)]),
    "hpvm_sgemm_tracked": (ctypes.c_int, [i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, i32,
                                          ctypes.POINTER(Tile), vp]),
    "hpvm_cpu_menu": (ctypes.c_int, [ctypes.POINTER(Tile), i32, ctypes.POINTER(i32)]),
    "hpvm_cpu_isa": (ctypes.c_char_p, []),
    "hpvm_sgemm_cpu": (ctypes.c_int, [i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64,
                                      ctypes.POINTER(Tile), i32]),
    "hpvm_stream_open": (ctypes.c_int, [ctypes.POINTER(StreamConfig), ctypes.POINTER(vp)]),
    "hpvm_stream_push": (ctypes.c_int, [vp, ctypes.POINTER(SgemmDesc), ctypes.POINTER(i64)]),
    "hpvm_stream_pop": (ctypes.c_int, [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(vp)]),
    "hpvm_stream_info": (ctypes.c_int, [vp, ctypes.POINTER(StreamStatus)]),
    "hpvm_stream_close": (ctypes.c_int, [vp, i32]),
}

_lib = None


def load(path: str | None = None):
    """Load (once) and return the ctypes library handle."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- binds the library to torch's HIP runtime

    # HPVM_SGEMM_LIB names another build of the same library (the tests'
    # sanitizer build of the host code).
    path = path or os.environ.get("HPVM_SGEMM_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
