"""MI355X-native LDG-Stokes multigrid V-cycle (Saye, arXiv:1911.05888).

The compute path is the C-ABI library ``libldgs.so`` (hand-written HIP
kernels for gfx950 plus C++ host setup); this package only binds it.
"""
from .ldgs import (Context, LdgsError, EXPORTED, LIB_PATH, TRAIN_WORKSPACE_BYTES, V_FP64, V_FP32, V_FP32_BF16BLK,  # noqa: F401
                   STATIONARY, IR, FGMRES, GMRES, learned_train, net_nparams, init_net_params)
