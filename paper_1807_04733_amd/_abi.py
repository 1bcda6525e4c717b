"""ctypes declarations of the libpic C ABI (include/pic.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpic.so")

MAX_LAYERS = 16
MAX_CHANNELS = 8
MAX_TTABLES = 8
MAX_TENTRIES = 64
MAX_EBINS = 128

F_STATE_FP64 = 1
F_SECONDARIES = 2
F_DEBUG = 4
F_GEN_MOMENT = 8
F_ABSORB_NEXT = 16
F_WEIGHTS = 32

COUNTER_NAMES = ("injected", "ev_ee", "ev_el", "spawned", "absorbed", "sec_absorbed",
                 "transmit", "refl_if", "refl_surf", "alive", "e_absorbed", "w_injected")
NCOUNTERS = len(COUNTER_NAMES)
STATIC_WORKSPACE_BYTES = 64 << 20   # PIC_STATIC_WORKSPACE_BYTES

STATUS = {0: "PIC_OK", 1: "PIC_EINVAL", 2: "PIC_ENOMEM", 3: "PIC_ECAPACITY", 4: "PIC_EHIP",
          5: "PIC_ESTATE"}

EXPORTS = ("pic_workspace_size", "pic_init", "pic_init_static", "pic_inject", "pic_step", "pic_compact", "pic_deposit",
           "pic_backward", "pic_counters", "pic_reset", "pic_set_tuning", "pic_get_tuning",
           "pic_layout_of", "pic_autotune", "pic_time_kernels", "pic_kernel_times",
           "pic_generations",
           "pic_destroy", "pic_last_error")


class PicInstance(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32), ("n_channels", C.c_int32), ("n_ttables", C.c_int32),
        ("t_entries", C.c_int32),
        ("z_bound", C.c_double * (MAX_LAYERS + 1)),
        ("ch_of", (C.c_int32 * 2) * MAX_LAYERS),
        ("v", C.c_double * MAX_CHANNELS),
        ("inv_tau0", C.c_double * MAX_CHANNELS),
        ("inv_tau_el", C.c_double * MAX_LAYERS),
        ("P0", C.c_double * MAX_LAYERS),
        ("tt_of", ((C.c_int32 * 2) * 2) * (MAX_LAYERS - 1)),
        ("T", (C.c_double * MAX_TENTRIES) * MAX_TTABLES),
        ("T_scale", C.c_double),
        ("src_z_lo", C.c_double), ("src_z_hi", C.c_double), ("src_lambda", C.c_double),
        ("src_cd", C.c_double), ("src_up_frac", C.c_double),
        ("src_e_lo", C.c_uint32 * 2), ("src_e_span", C.c_uint32 * 2),
        ("n_primaries", C.c_int64), ("root_offset", C.c_uint64),
        ("nz", C.c_int32), ("inv_dz", C.c_double),
        ("e_nodes", C.c_int32), ("e_scale", C.c_double),
        ("v_node", (C.c_double * MAX_TENTRIES) * MAX_CHANNELS),
        ("r_node", (C.c_double * MAX_TENTRIES) * MAX_CHANNELS),
        ("w_nodes", C.c_int32), ("w_scale", C.c_double),
        ("w_node", (C.c_double * MAX_TENTRIES) * 2),
    ]


class PicConfig(C.Structure):
    _fields_ = [
        ("n_instances", C.c_int32), ("inst", C.POINTER(PicInstance)), ("seed", C.c_uint64),
        ("dt", C.c_double), ("n_steps", C.c_int32), ("tau_exp", C.c_int32),
        ("e_min_fx", C.c_uint32), ("flags", C.c_uint32), ("n_ebins", C.c_int32),
        ("e_edges", C.c_uint32 * MAX_EBINS), ("dens_stride", C.c_int32),
        ("cur_stride", C.c_int32), ("slab_primaries", C.c_int32),
        ("capacity_factor", C.c_double), ("adjoint", C.c_int32),
    ]


class PicTuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("grid", C.c_int32), ("compact_every", C.c_int32),
                ("compact_frac", C.c_float), ("use_graph", C.c_int32), ("z_every", C.c_int32),
                ("sub_steps", C.c_int32)]


class PicLayout(C.Structure):
    _fields_ = [
        ("n_slabs", C.c_int64), ("capacity", C.c_int64),
        ("off_z", C.c_int64), ("off_mu", C.c_int64), ("off_E", C.c_int64),
        ("off_uid", C.c_int64), ("off_flags", C.c_int64), ("off_ev", C.c_int64),
        ("off_slab_base", C.c_int64), ("off_slab_cap", C.c_int64),
        ("off_slab_tail", C.c_int64), ("off_slab_dead", C.c_int64),
        ("off_slab_inst", C.c_int64),
        ("off_dens", C.c_int64), ("off_cur", C.c_int64), ("off_counters", C.c_int64),
        ("dens_len", C.c_int64), ("cur_len", C.c_int64),
        ("state_bytes", C.c_int32), ("flags_spin_shift", C.c_int32),
        ("flags_layer_shift", C.c_int32), ("flags_layer_bits", C.c_int32),
        ("flags_gen_shift", C.c_int32), ("flags_dead_bit", C.c_uint32),
        ("off_w", C.c_int64),
    ]


_lib = None


def load():
    """Load libpic.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    sig = {
        "pic_workspace_size": ([P(PicConfig), P(C.c_int64)], C.c_int),
        "pic_init": ([P(PicConfig), vp, C.c_int64, vp, P(vp)], C.c_int),
        "pic_init_static": ([P(PicConfig), vp, P(vp)], C.c_int),
        "pic_inject": ([vp, P(C.c_int64)], C.c_int),
        "pic_step": ([vp, C.c_int32], C.c_int),
        "pic_compact": ([vp], C.c_int),
        "pic_deposit": ([vp, vp, vp], C.c_int),
        "pic_backward": ([vp, vp, vp, vp, C.c_int32], C.c_int),
        "pic_counters": ([vp, P(C.c_int64)], C.c_int),
        "pic_reset": ([vp], C.c_int),
        "pic_set_tuning": ([vp, P(PicTuning)], C.c_int),
        "pic_get_tuning": ([vp, P(PicTuning)], C.c_int),
        "pic_layout_of": ([vp, P(PicLayout)], C.c_int),
        "pic_autotune": ([vp, C.c_int32, P(PicTuning)], C.c_int),
        "pic_time_kernels": ([vp, C.c_int32], C.c_int),
        "pic_generations": ([vp, vp], C.c_int),
        "pic_kernel_times": ([vp, P(C.c_double), C.c_int32, P(C.c_int32)], C.c_int),
        "pic_destroy": ([vp], None),
        "pic_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def check(code):
    if code != 0:
        msg = load().pic_last_error().decode(errors="replace")
        raise PicError(code, msg)
