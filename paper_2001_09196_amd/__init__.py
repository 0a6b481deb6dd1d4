"""MI355X (gfx950) S_N source iteration with heterogeneous (thick-only) DSA.

The compute path is libsn.so (HIP kernels behind the C ABI of include/sn.h);
`binding` marshals torch device tensors into it and `adjoint` wraps the
adjoint gradient in a torch.autograd.Function.  Nothing here falls back to
the CPU: without the built library the binding raises.
"""
from . import binding  # noqa: F401
from .binding import (SN_DIFFUSION_MNIP, SN_DIFFUSION_NIP, SN_DIFFUSION_SIP, SN_DSA_DIAGONAL,  # noqa: F401
                      SN_DSA_TRIANGULAR, SN_FP32, SN_FP64, SN_PRECOND_BLOCK_JACOBI, SN_PRECOND_DIRECT,
                      SN_PRECOND_MG, Context, SnError, sn_adjoint_gradient, sn_adjoint_source, sn_dsa_thick_correct,
                      sn_face_response, sn_gradient, sn_kernel_timing, sn_krylov_solve, sn_response, sn_response_noalloc,
                      sn_scalar_flux,
                      sn_set_kernel_timing, sn_source_iterate, sn_sweep)
