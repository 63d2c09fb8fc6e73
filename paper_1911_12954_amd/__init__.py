"""HOTRG and ATRG coarse-graining of the Ising tensor network on AMD MI355X (gfx950).

The computation lives in the HIP library ``libtrg.so`` (C-ABI declared in
``include/trg.h``); ``trg`` is its Python binding.  Build the library with
``python -m paper_1911_12954_amd.build``.
"""
from .trg import (Context, TrgError, trg_atrg_step, trg_eigh, trg_eigh_top, trg_eigh_top_work_bytes,  # noqa: F401
                  trg_export_state, trg_footprint_bytes,
                  trg_free_energy, trg_gemm, trg_gemm_tile, trg_hotrg_step, trg_hotrg_step_batch,
                  trg_import_state, trg_impure_energy,
                  trg_impure_magnetization, trg_indicator_x, trg_init_factors, trg_init_ising, trg_init_tensor,
                  trg_resident_bytes, trg_run, trg_share_workspace, trg_workspace_bytes)
