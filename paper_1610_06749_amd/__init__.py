"""MI355X-native recombination solver (IonTracks method, arXiv:1610.06749).

The solver is the HIP library ``libiontracks.so`` (C ABI in
``include/iontracks.h``); ``binding`` marshals Python arguments to it.  There
is no CPU fallback: the entry points raise if the library is not built or
no GPU is present.
"""
from .binding import (IT_EHIP, IT_EINVAL, IT_ENODT, IT_ENOTSUP, IT_EWORKSPACE, IT_FLAG_EMPTY,  # noqa: F401
                      IT_FLAG_MAX_STEPS, IT_FLAG_NONFINITE, IT_FLAG_REACTION, IT_KERNEL_AUTO,
                      IT_KERNEL_BLOCKED, IT_KERNEL_PLAIN, IT_OK, IT_TRACE_COLS, TRACE_KEYS, ItError,
                      it_advance, it_dt, it_solve, it_solve_batch, it_strerror, it_validate, it_workspace_size,
                      it_workspace_size_batch, lib, IT_MLP_PARAMS, IT_MLP_BF16, IT_MLP_FP32, it_mlp_model_bytes, it_mlp_init,
                      it_mlp_grad, it_mlp_train, it_mlp_query, it_mlp_baseline,
                      it_mlp_query_static, IT_MLP_QUERY_STATIC_MAX, it_host_buffer_size, host_buffer,
                      workspace, KernelTimer)
