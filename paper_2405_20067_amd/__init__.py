"""MI355X-native evaluation and differentiation of N-D Gaussian mixtures
with random-projection tile culling (Diolatzis et al., "N-Dimensional
Gaussians for Fitting of High Dimensional Functions", SIGGRAPH 2024).

The compute path is the HIP library libngd.so (C-ABI, include/ngd.h);
`paper_2405_20067_amd.ngd` is its thin Python binding and
`paper_2405_20067_amd.autograd` the torch.autograd wrapper.  Importing this
package loads nothing; the library is loaded on first use and a missing
library is an error.
"""

__all__ = ["inputs"]
