"""MI355X (gfx950) implementation of the EOS-based pseudo-potential lattice Boltzmann step with the geometric
contact-angle wall of Hu, Li & Uddin (arXiv:1501.05430). The method runs in liblbm.so (HIP kernels behind the
C-ABI of include/lbm.h); this package only marshals arguments and lends torch's device memory and streams."""
from ._lib import LbmError, Params, load  # noqa: F401
from .lbm import LBM, eos_coexistence, fp32_options, make_params, workspace_bytes  # noqa: F401
