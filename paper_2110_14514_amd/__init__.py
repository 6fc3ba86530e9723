"""gcpstream: streaming GCP objective and gradient on MI355X.

The computation lives in the HIP library libgcpstream.so (C ABI in
include/gcpstream.h); this package marshals arguments to it and supplies
device memory and streams through PyTorch.
"""
from . import _native  # noqa: F401
from .autograd import GcpLoss, gcp_loss  # noqa: F401
from .stream import (Batch, Stream, gcp_loss_grad, gcp_solve_st, gcp_stream_init,  # noqa: F401
                     gcp_update_factors, gcp_workspace_size, make_params)

__all__ = ["Batch", "GcpLoss", "gcp_loss", "Stream", "gcp_stream_init", "gcp_loss_grad", "gcp_solve_st",
           "gcp_update_factors", "gcp_workspace_size", "make_params"]
