"""ctypes view of libim.so (the C ABI declared in include/im.h).

Argument marshalling only: every step of the selection runs in the HIP
kernels behind these entry points. There is no fallback; if the library is
missing the import fails.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libim.so")

IM_OK, IM_EINVAL, IM_EOVERFLOW, IM_ENOMEM, IM_EHIP = 0, -1, -2, -3, -4
IM_R_MAX = 4096

EXPORTS = ("im_workspace_create", "im_workspace_destroy", "im_stats_get", "im_last_error",
           "im_validate", "im_snapshot_masks", "im_transpose", "im_initial_gains", "im_select",
           "im_profile_enable", "im_profile_get", "im_workspace_set", "im_profile_launches",
           "im_plan_create", "im_plan_launch", "im_plan_stats", "im_plan_destroy",
           "im_select_batch", "im_mlp_create", "im_mlp_destroy", "im_mlp_set_params",
           "im_mlp_get_params", "im_mlp_forward", "im_mlp_loss_grad", "im_mlp_adam",
           "im_mlp_train_step", "im_node_features", "im_mlp_samples", "im_select_lazy",
           "im_autotune", "im_autotune_batch", "im_plan_create_batch", "im_spread",
           "im_pair_ids", "im_select_undirected", "im_select_noalloc", "im_autotune_lazy")
IM_MLP_NPARAM = 4609
IM_SPREAD_R_MAX = 1 << 20
IM_PH_MAX = 24
IM_NOALLOC_SCRATCH_BYTES = 128 << 20

PHASES = ("validate", "transpose", "mask_gen", "mask_gather", "init_t0", "init_t1", "init_t2",
          "argmax", "forward", "rev_t0", "rev_t1", "rev_t2", "clear", "call", "hubs",
          "pack", "order", "score", "pick", "eval_t0", "eval_t1", "eval_t2", "update", "affected")
IM_OPT_HUB_DEGREE = 1
IM_OPT_COOP_GAIN = 2
IM_OPT_LAZY_ENGINE = 3
IM_OPT_MAX_SLOTS = 4
IM_OPT_TIER1_SHAPE = 5
IM_OPT_TIER2_LANES = 6
IM_OPT_SPARSE_LISTS = 7
IM_OPT_FWD_GROUPS = 8
IM_OPT_LEARNED_POLICY = 9
IM_OPT_PAIR_COINS = 10
IM_OPT_LIVE_EDGE = 11
IM_OPT_LAZY_BATCH = 12
IM_OPT_AFFECTED_GAIN = 13
IM_OPT_EVAL_SPLIT = 14
IM_OPT_REV_SPLIT = 15
IM_OPT_REV_FIRST_TIER = 16


class ImGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("prob", ctypes.c_void_p)]


class ImInstance(ctypes.Structure):
    _fields_ = [("g", ImGraph), ("R", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("seed", ctypes.c_uint64)]


STAT_FIELDS = ("trav_init", "trav_fwd", "trav_rev", "trav_eval", "relax_fwd", "tasks_rev",
               "decrements", "celf_evals")
PASSES = ("init", "rev", "eval")
TIER_FIELDS = ("relax", "reached", "arcs_read", "handed_over")


class ImStats(ctypes.Structure):
    _fields_ = ([(f, ctypes.c_uint64) for f in STAT_FIELDS] +
                [(f, (ctypes.c_uint64 * 3) * 3) for f in TIER_FIELDS] +
                [("fwd_levels", ctypes.c_uint64), ("fwd_entries", ctypes.c_uint64),
                 ("celf_batches", ctypes.c_uint64), ("celf_fallbacks", ctypes.c_uint64),
                 ("max_levels", (ctypes.c_uint64 * 3) * 3),
                 ("barrier_failures", ctypes.c_uint64),
                 ("reserved", ctypes.c_uint64 * 6)])

    def as_dict(self):
        d = {f: int(getattr(self, f)) for f in STAT_FIELDS + ("fwd_levels", "fwd_entries",
                                                               "celf_batches", "celf_fallbacks",
                                                               "barrier_failures")}
        for p, pn in enumerate(PASSES):
            for t in range(3):
                d[f"max_levels_{pn}_t{t}"] = int(self.max_levels[p][t])
        for f in TIER_FIELDS:
            arr = getattr(self, f)
            for p, pn in enumerate(PASSES):
                per = [int(arr[p][t]) for t in range(3)]
                d[f"{f}_{pn}"] = sum(per)
                for t in range(3):
                    d[f"{f}_{pn}_t{t}"] = per[t]
        return d


class ImTuning(ctypes.Structure):
    _fields_ = [("hub_degree", ctypes.c_int32), ("tier1_shape", ctypes.c_int32),
                ("tier2_lanes", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("coop_forward", ctypes.c_int32), ("ms", ctypes.c_float), ("tried", ctypes.c_uint32),
                ("affected_gain", ctypes.c_uint64), ("fwd_groups", ctypes.c_int32),
                ("rev_split", ctypes.c_int32), ("rev_first_tier", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ImLazyTuning(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_int32), ("batch", ctypes.c_uint32), ("ms", ctypes.c_float),
                ("tried", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ImProfile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * IM_PH_MAX), ("launches", ctypes.c_uint64 * IM_PH_MAX)]


class ImError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libim error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (paper_1212_4779_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        p, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        G = ctypes.POINTER(ImGraph)
        L.im_workspace_create.argtypes = [ctypes.POINTER(p)]
        L.im_workspace_destroy.argtypes = [p]
        L.im_stats_get.argtypes = [p, ctypes.POINTER(ImStats)]
        L.im_last_error.restype = ctypes.c_char_p
        L.im_validate.argtypes = [G, u32, p]
        L.im_snapshot_masks.argtypes = [G, u32, u64, p, p, p]
        L.im_transpose.argtypes = [G, p, p, p, p, p]
        L.im_initial_gains.argtypes = [G, u32, u64, p, p, p]
        L.im_select.argtypes = [G, u32, u32, u64, p, p, p, p, p]
        L.im_profile_enable.argtypes = [p, u32]
        L.im_workspace_set.argtypes = [p, ctypes.c_int, ctypes.c_int64]
        L.im_profile_launches.argtypes = [p, ctypes.c_int, p, u32, ctypes.POINTER(u32)]
        L.im_plan_create.argtypes = [G, u32, u32, u64, p, p, p, ctypes.POINTER(p)]
        L.im_plan_launch.argtypes = [p, p]
        L.im_plan_stats.argtypes = [p, ctypes.POINTER(ImStats)]
        L.im_plan_destroy.argtypes = [p]
        L.im_select_batch.argtypes = [ctypes.POINTER(ImInstance), u32, p, p, p, p]
        L.im_profile_get.argtypes = [p, ctypes.POINTER(ImProfile)]
        f32 = ctypes.c_float
        L.im_mlp_create.argtypes = [ctypes.POINTER(p)]
        L.im_mlp_destroy.argtypes = [p]
        L.im_mlp_set_params.argtypes = [p, p]
        L.im_mlp_get_params.argtypes = [p, p, p]
        L.im_mlp_forward.argtypes = [p, p, u32, p, p]
        L.im_mlp_loss_grad.argtypes = [p, p, p, u32, p, p, p]
        L.im_mlp_adam.argtypes = [p, p, f32, f32, f32, f32, p]
        L.im_mlp_train_step.argtypes = [p, p, p, u32, p, u32, p, p, f32, f32, f32, f32, p]
        L.im_node_features.argtypes = [G, p, p, p]
        L.im_mlp_samples.argtypes = [p, p, u32, u32, u32, p, p, p, u32, p, p, p]
        L.im_select_lazy.argtypes = [G, u32, u32, u64, u32, p, p, p, p, p]
        L.im_autotune.argtypes = [G, u32, u64, p, p, ctypes.POINTER(ImTuning)]
        L.im_autotune_batch.argtypes = [ctypes.POINTER(ImInstance), u32, p, p, ctypes.POINTER(ImTuning)]
        L.im_plan_create_batch.argtypes = [ctypes.POINTER(ImInstance), u32, p, p, p, p, ctypes.POINTER(p)]
        L.im_spread.argtypes = [G, u32, u64, p, u32, p, p, p, p]
        L.im_pair_ids.argtypes = [G, p, p, p]
        L.im_select_undirected.argtypes = [G, u32, u32, u64, p, p, p, p, p]
        L.im_select_noalloc.argtypes = [G, u32, u32, u64, p, p, p]
        L.im_autotune_lazy.argtypes = [G, u32, u32, u64, p, p, p, ctypes.POINTER(ImLazyTuning)]
        for name in EXPORTS:
            getattr(L, name).restype = ctypes.c_int if name != "im_last_error" else ctypes.c_char_p
        _lib = L
    return _lib


def check(rc):
    if rc != IM_OK:
        raise ImError(rc, lib().im_last_error().decode())
