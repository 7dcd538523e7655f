"""FP64 CPU oracle for the feature-distilled Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import this package.  The product path
(the HIP library and its Python binding) never imports, calls or links
anything here; the two share no code.

Every function follows the paper's definitions in plain PyTorch CPU float64:
* eq. (1)  Gaussian falloff exp(-1/2 d^T Sigma^-1 d), evaluated in 2-D;
* eq. (2)  Sigma = R S S^T R^T;
* eq. (9)  Sigma' = J W Sigma W^T J^T (affine approximation of projection);
* eqs. (7)-(8) front-to-back blending of colour and semantic features with
  the same weights alpha_i prod_{j<i} (1 - alpha_j);
* eq. (10) the pointwise-convolution decoder and its per-pixel L1 loss;
* eqs. (4)-(6) the FST deformation module (HexPlane, F_out, the four
  branches and the semantic updater) that produces G_t.
The discrete rules the paper leaves open (tile binning, alpha clamp, skip and
stop thresholds, SH convention, pixel centres) are the readings listed in the
design notes; each is restated where it is used.

The backward pass is the derivative of this forward as written (torch
autograd over the same float64 graph, tile by tile), pinned by central finite
differences in the tests.
"""
from .sh import sh_basis, sh_coeff_count
from .project import project, OracleCamera, OracleConfig
from .raster import (bin_gaussians, composite, render_forward, brute_force_render,
                     TileLists)
from .grad import render_backward, fd_gradient
from .decoder import decoder_l1
from .deform import deform_gaussians, hexplane_features, deform_mlp

__all__ = ["sh_basis", "sh_coeff_count", "project", "OracleCamera", "OracleConfig",
           "bin_gaussians", "composite", "render_forward", "brute_force_render",
           "TileLists", "render_backward", "fd_gradient", "decoder_l1", "deform_gaussians", "hexplane_features",
           "deform_mlp"]
