"""MI355X (gfx950) primal-dual symmetric-cone MWU for the smallest enclosing
sphere and hard-margin SVM problems (Zheng, Varvitsiotis, Tan, Lin,
arXiv 2405.09157).

The compute path is the HIP library ``libscpmwu.so`` behind the C ABI of
``include/scp_mwu.h``; this package only marshals arguments to it.  torch is
used for device memory and streams.

    import torch, paper_2405_09157_amd as scp
    X = torch.randn(1_000_000, 100, device="cuda")
    with scp.MWU(X, problem="ses") as m:
        out = m.solve()              # radius, centre, certified bounds
"""
from __future__ import annotations

from ._lib import (  # noqa: F401  (re-exported C-ABI names)
    EXPORTS, OUTCOME_NAMES, SCP_MWU_BF16, SCP_MWU_E_HIP, SCP_MWU_E_INFEASIBLE, SCP_MWU_E_INVAL,
    SCP_MWU_E_NOMEM, SCP_MWU_E_NUMERIC, SCP_MWU_E_STATE, SCP_MWU_E_UNSUPPORTED, SCP_MWU_F32, SCP_MWU_F64, SCP_MWU_FP8,
    SCP_MWU_OK, SCP_MWU_STOPPED,
    SCP_MWU_FLAG_CERTIFICATES, SCP_MWU_FLAG_DETERMINISTIC, SCP_MWU_FLAG_NO_EARLY_STOP, SCP_MWU_FLAG_THEORY,
    SCP_MWU_PROBLEM_SES, SCP_MWU_PROBLEM_SVM, ScpMwuError, load, scp_mwu_backward,
    scp_mwu_cast_bf16, scp_mwu_desc, scp_mwu_destroy, scp_mwu_get_D, scp_mwu_get_state,
    scp_mwu_get_vector, scp_mwu_init, scp_mwu_result, scp_mwu_set_state, scp_mwu_solve,
    scp_mwu_quantize_fp8, scp_mwu_product_exp, scp_mwu_product_init, scp_mwu_product_destroy, scp_mwu_read_reference, scp_mwu_step, scp_mwu_stepinfo, scp_mwu_strerror, scp_mwu_time_passes,
    scp_mwu_batch_desc, scp_mwu_batch_destroy, scp_mwu_batch_get_D, scp_mwu_batch_get_vector, scp_mwu_batch_init,
    scp_mwu_batch_solve, scp_mwu_batch_solve_kway, scp_mwu_batch_step, scp_mwu_batch_time_iters)
from .api import MWU, MWUBatch, ProductCone, autotune_rows_per_group, product_exp, ses_radius  # noqa: F401
