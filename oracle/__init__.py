"""FP64 CPU oracle for the TensorNet energy-and-forces path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library (no kernels, headers, helpers, constants or pre/post
processing): it reads the same weight blob with its own parser and takes the
same seeded inputs from `synth`, nothing else.

Contents
  blob       independent parser of the weight blob
  neighbors  O1: unordered pair set {i<j, same system, d^2 < r_c^2} with the
             minimum image in a rectangular or triclinic cell (brute force +
             a CPU cell list)
  model      O2-O6: geometry, exp-normal basis, cosine cutoff, embedding,
             interaction layers, output network, energies, and forces by
             torch.autograd, all in float64 on full 3x3 matrices
  train      the energy + force loss and its parameter gradient by torch
             double autograd (the training step's reference)

Every function cites the part of the paper it follows (TorchMD-Net 2.0,
arXiv 2402.17660): the TensorNet paragraph of Sec. 2.1.1, the hyper-parameter
listing of Sec. 2.4, the neighbour-search discussion of Sec. 2.5.1 and
Tables S3/S4.  Where the paper is silent the reading adopted is stated next to
the code.  Parity with the published TensorNet numerics is unpinned: the paper
prints no worked example or intermediate value for it.
"""

from .blob import read_blob  # noqa: F401
from .neighbors import neighbor_pairs, brute_force_pairs, cell_list_pairs  # noqa: F401
from .model import (  # noqa: F401
    TensorNetOracle,
    decompose,
    symmetric_product,
    mix,
    tensor_norm,
    skew,
    sym_traceless_outer,
    cosine_cutoff,
    expnorm_constants,
    expnorm_rbf,
    layer_norm,
    silu,
)
from .train import training_loss, training_loss_and_grad  # noqa: F401,E402
