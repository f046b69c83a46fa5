"""ctypes binding of libpcmcc.so (the C ABI declared in include/pcmcc.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch tensors provide device memory and streams.  If the built
library is missing the import fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcmcc.so")

PCMCC_OK, PCMCC_EINVAL, PCMCC_ECAPACITY, PCMCC_EHIP = 0, -1, -2, -3
PCMCC_ESTATE, PCMCC_ENOMEM, PCMCC_ETABLE, PCMCC_ELIMIT, PCMCC_ERANGE = -4, -5, -6, -7, -8
PCMCC_ELASTIC, PCMCC_EXCITATION, PCMCC_IONIZATION, PCMCC_ATTACHMENT = 0, 1, 2, 3
PCMCC_EFFECTIVE_TO_ELASTIC, PCMCC_RATES = 1, 2

_NAMES = {0: "OK", -1: "EINVAL", -2: "ECAPACITY", -3: "EHIP", -4: "ESTATE", -5: "ENOMEM", -6: "ETABLE",
          -7: "ELIMIT", -8: "ERANGE"}


class pcmcc_particles(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("vx", C.c_void_p),
                ("vy", C.c_void_p), ("vz", C.c_void_p), ("w", C.c_void_p), ("id", C.c_void_p),
                ("n_dev", C.c_void_p), ("capacity", C.c_int64)]


class pcmcc_grid(C.Structure):
    _fields_ = [("E", C.c_void_p), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("x0", C.c_double),
                ("y0", C.c_double), ("z0", C.c_double), ("dx", C.c_double)]


class pcmcc_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("steps_done", C.c_int64), ("particle_steps", C.c_uint64),
                ("trials", C.c_uint64), ("null_collisions", C.c_uint64),
                ("real_collisions", C.c_uint64 * 4), ("lost", C.c_uint64), ("out_of_table", C.c_uint64),
                ("errors", C.c_uint64), ("step_kernel_ms", C.c_double), ("deposit_kernel_ms", C.c_double),
                ("launch_block", C.c_int32), ("launch_grid", C.c_int32), ("weight_updates", C.c_int64),
                ("merged_pairs", C.c_int64), ("splits", C.c_int64), ("weight_ms", C.c_double),
                ("field_ms", C.c_double), ("mg_cycles", C.c_int64), ("photons", C.c_int64),
                ("photoelectrons", C.c_int64), ("photo_ms", C.c_double), ("majorant_violations", C.c_uint64),
                ("launch_refill", C.c_int32), ("launch_chunk", C.c_int32)]

    def as_dict(self) -> dict:
        r = list(self.real_collisions)
        return {"n": self.n, "steps_done": self.steps_done, "particle_steps": self.particle_steps,
                "trials": self.trials, "null": self.null_collisions, "elastic": r[0], "excitation": r[1],
                "ionization": r[2], "attachment": r[3], "lost": self.lost,
                "out_of_table": self.out_of_table, "errors": self.errors,
                "step_kernel_ms": self.step_kernel_ms, "deposit_kernel_ms": self.deposit_kernel_ms,
                "launch_block": self.launch_block, "launch_grid": self.launch_grid,
                "weight_updates": self.weight_updates, "merged_pairs": self.merged_pairs, "splits": self.splits,
                "weight_ms": self.weight_ms, "field_ms": self.field_ms, "mg_cycles": self.mg_cycles,
                "photons": self.photons, "photoelectrons": self.photoelectrons, "photo_ms": self.photo_ms,
                "majorant_violations": self.majorant_violations, "launch_refill": self.launch_refill,
                "launch_chunk": self.launch_chunk}


class pcmcc_schedule(C.Structure):
    _fields_ = [("block", C.c_int), ("blocks_per_cu", C.c_int), ("refill_min", C.c_int), ("chunk", C.c_int)]

    def as_dict(self) -> dict:
        return {"block": self.block, "blocks_per_cu": self.blocks_per_cu, "refill_min": self.refill_min,
                "chunk": self.chunk}


SWARM_QUANTITIES = ("W_flux", "W_bulk", "DL_flux", "DL_bulk", "DT_flux", "DT_bulk", "nu_ion", "nu_att",
                    "nu_eff", "mean_eps", "mu", "alpha", "eta", "bulk_flux_ratio")
SWARM_NQ = len(SWARM_QUANTITIES)
SWARM_NMOM = 14


class pcmcc_photo_opts(C.Structure):
    _fields_ = [("eta", C.c_double), ("k1", C.c_double), ("k2", C.c_double), ("w_photon", C.c_double)]


class pcmcc_sc_opts(C.Structure):
    _fields_ = [("adaptive", C.c_int), ("dt_max", C.c_double), ("cfl", C.c_double), ("growth_max", C.c_double),
                ("mu_n", C.c_int), ("mu_EN_lo", C.c_double), ("mu_EN_hi", C.c_double), ("mu_N", C.c_void_p),
                ("mg_tol", C.c_double), ("mg_max_cycles", C.c_int), ("photo", C.POINTER(pcmcc_photo_opts))]


class pcmcc_fluid_table(C.Structure):
    _fields_ = [("n", C.c_int), ("EN_lo", C.c_double), ("EN_hi", C.c_double), ("muN", C.c_void_p),
                ("DN", C.c_void_p), ("alphaN", C.c_void_p), ("etaN", C.c_void_p)]


class pcmcc_swarm_opts(C.Structure):
    _fields_ = [("sample_every", C.c_int), ("window_start_s", C.c_double), ("n_batches", C.c_int),
                ("cap_factor", C.c_int), ("population_control", C.c_int), ("block", C.c_int),
                ("blocks_per_cu", C.c_int), ("autotune", C.c_int), ("tune_cache", C.c_char_p),
                ("refill_min", C.c_int), ("chunk", C.c_int)]


class pcmcc_swarm_result(C.Structure):
    _fields_ = [("value", C.c_double * SWARM_NQ), ("error", C.c_double * SWARM_NQ)]


MLP_PARAMS = 4678
MLP_OUT = 6


class pcmcc_mlp_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int), ("lr0", C.c_double), ("lr_min", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double)]


class pcmcc_mlp_infer_opts(C.Structure):
    _fields_ = [("mu_x", C.c_double), ("sd_x", C.c_double), ("mu_y", C.c_double * MLP_OUT),
                ("sd_y", C.c_double * MLP_OUT), ("n_cells", C.c_int), ("cell_lo", C.c_double),
                ("cell_hi", C.c_double), ("fallback", C.c_void_p), ("n_nodes", C.c_int),
                ("table_lo", C.c_double), ("table_hi", C.c_double), ("table", C.c_void_p)]


class PcmccError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pcmcc error {code} ({_NAMES.get(code, '?')}): {msg}")
        self.code = code


_lib = None


def lib() -> C.CDLL:
    """Loads libpcmcc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2110_14494_amd/build.py "
                              "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i64, u64 = C.c_void_p, C.c_int64, C.c_uint64
        sigs = {
            "pcmcc_version": ([], C.c_char_p),
            "pcmcc_last_error": ([vp], C.c_char_p),
            "pcmcc_create": ([C.POINTER(vp), C.c_int, vp], C.c_int),
            "pcmcc_destroy": ([vp], C.c_int),
            "pcmcc_init_species": ([vp, C.c_double, C.c_double, C.c_double, C.c_double], C.c_int),
            "pcmcc_init_tables": ([vp, C.c_int, C.c_double, C.c_double, C.c_int, vp, vp, vp, C.c_int], C.c_int),
            "pcmcc_push_collide_deposit": ([vp, C.POINTER(pcmcc_particles), C.POINTER(pcmcc_grid), C.c_double,
                                            C.c_int, u64, u64, vp, C.POINTER(pcmcc_stats)], C.c_int),
            "pcmcc_set_schedule": ([vp, C.POINTER(pcmcc_schedule)], C.c_int),
            "pcmcc_get_schedule": ([vp, C.POINTER(pcmcc_schedule)], C.c_int),
            "pcmcc_autotune_steps": ([vp, C.POINTER(pcmcc_particles), C.POINTER(pcmcc_grid), C.c_double, C.c_int,
                                      u64, u64, C.c_char_p, C.POINTER(pcmcc_schedule), C.POINTER(C.c_float),
                                      C.POINTER(C.c_float)], C.c_int),
            "pcmcc_deposit": ([vp, vp, vp, vp, vp, vp, C.POINTER(pcmcc_grid), vp], C.c_int),
            "pcmcc_deposit_noalloc": ([vp, vp, vp, vp, vp, vp, C.POINTER(pcmcc_grid), vp], C.c_int),
            "pcmcc_philox4x32_10": ([vp, i64, vp, u64, vp], C.c_int),
            "pcmcc_tables_lookup": ([vp, i64, vp, vp, vp, vp], C.c_int),
            "pcmcc_mlp_grad": ([vp, vp, i64, vp, vp, vp, vp, C.POINTER(C.c_double)], C.c_int),
            "pcmcc_mlp_train": ([vp, vp, i64, vp, vp, vp, C.POINTER(pcmcc_mlp_train_opts), vp, vp,
                                 C.POINTER(pcmcc_stats)], C.c_int),
            "pcmcc_mlp_infer": ([vp, vp, C.POINTER(pcmcc_mlp_infer_opts), i64, vp, vp, C.POINTER(pcmcc_stats)],
                                C.c_int),
            "pcmcc_mlp_dataset": ([C.c_int, vp, vp, C.c_double, C.c_double, C.c_int,
                                   C.POINTER(pcmcc_mlp_infer_opts), vp, vp, vp, vp, vp, C.c_double], C.c_int),
            "pcmcc_mlp_fallback": ([vp, vp, C.POINTER(pcmcc_mlp_infer_opts), C.c_int, vp, vp, vp, vp, C.c_double,
                                    C.c_double, C.c_int, C.c_double, C.c_double, vp, vp], C.c_int),
            "pcmcc_set_weight_control": ([vp, C.c_double, C.c_double], C.c_int),
            "pcmcc_update_weights": ([vp, C.POINTER(pcmcc_particles), C.POINTER(pcmcc_grid), C.c_double, u64, u64,
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
            "pcmcc_solve_potential": ([vp, C.POINTER(pcmcc_grid), vp, vp, vp, vp, C.c_double, C.c_int,
                                       C.POINTER(C.c_int), C.POINTER(C.c_double)], C.c_int),
            "pcmcc_field_from_potential": ([vp, C.POINTER(pcmcc_grid), vp, vp], C.c_int),
            "pcmcc_speed_quantile": ([vp, vp, vp, vp, vp, C.POINTER(C.c_double)], C.c_int),
            "pcmcc_streamer_steps": ([vp, C.POINTER(pcmcc_particles), C.POINTER(pcmcc_grid), vp, vp, vp, vp,
                                      C.POINTER(pcmcc_sc_opts), C.c_int, u64, u64, C.POINTER(C.c_double), vp,
                                      C.POINTER(pcmcc_stats)], C.c_int),
            "pcmcc_photoionize": ([vp, C.POINTER(pcmcc_grid), vp, vp, vp, vp, i64, C.POINTER(pcmcc_photo_opts), u64,
                                   u64, C.POINTER(pcmcc_particles), vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
                                  C.c_int),
            "pcmcc_fluid_steps": ([vp, C.POINTER(pcmcc_grid), vp, vp, vp, vp, C.POINTER(pcmcc_fluid_table), C.c_double,
                                   C.c_double, C.c_int, C.c_int, vp, vp, C.POINTER(pcmcc_stats)], C.c_int),
            "pcmcc_swarm_batch": ([vp, C.c_int, vp, vp, C.c_double, C.c_int, u64, C.POINTER(pcmcc_swarm_opts),
                                   vp, vp, vp, C.POINTER(pcmcc_stats)], C.c_int),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(rc: int, ctx=None) -> int:
    if rc != PCMCC_OK:
        raise PcmccError(rc, lib().pcmcc_last_error(ctx).decode())
    return rc
