"""MI355X (gfx950) GRMHD zone-update library: thin Python binding of libgrmhd.so.

Every step of the method runs in the HIP kernels of ``libgrmhd.so``; this
module only marshals arguments (problem struct, device pointers from torch
tensors, the current HIP stream). The functions carry the C ABI's names
(``grmhd_init``, ``grmhd_prim_to_cons``, ``grmhd_cons_to_prim``,
``grmhd_get_dt``, ``grmhd_step``, ``grmhd_divb``, ...); ``Sim`` is a small
convenience wrapper around them.

Importing never falls back to anything: if the library is missing the import
raises, and every call raises ``GrmhdError`` on a non-zero status.
"""

from ._binding import (  # noqa: F401
    GrmhdError, Problem, LIB_PATH, lib, NG, NVAR,
    GRMHD_OK, GRMHD_EINVAL, GRMHD_ENOMEM, GRMHD_EDEVICE, GRMHD_EUNSUPPORTED, GRMHD_ESTATE,
    GRMHD_OPT_FLOORS, GRMHD_OPT_FIXUP, EXPORTED, NSCALAR, HEAT_MODELS,
    grmhd_init, grmhd_free, grmhd_state_layout, grmhd_prim_to_cons, grmhd_cons_to_prim,
    grmhd_get_dt, grmhd_step, grmhd_step_electrons, grmhd_run_electrons, grmhd_run, grmhd_fill_ghosts, grmhd_substep, grmhd_update, grmhd_fixup, grmhd_speeds, grmhd_courant_dt,
    grmhd_divb, grmhd_divb_noalloc, grmhd_step_failures, grmhd_strerror,
    grmhd_last_error, grmhd_version, grmhd_profile, grmhd_profile_kernels, grmhd_profile_read, KERNELS, Sim,
    grmhd_set_tiles, grmhd_get_tiles, TILES, grmhd_context_bytes,
    grmhd_batch_create, grmhd_batch_set_dt, grmhd_batch_get, grmhd_batch_step, grmhd_batch_step_electrons,
    grmhd_batch_free,
    grmhd_batch_last_error, grmhd_batch_profile, grmhd_batch_profile_read, Batch,
)
