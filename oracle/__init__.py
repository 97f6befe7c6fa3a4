"""Plain FP64 CPU oracle of the CTD Allen-Cahn step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the package's smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
(the only common module is the seeded input generator `workloads`, which
holds none of the method's arithmetic).

Every routine follows the paper (Lu, Yuan, Guo, "Convolution tensor
decomposition for efficient high-resolution solutions to the Allen-Cahn
equation", arXiv 2410.15519) in its order and notation; each function cites
the section / equation it implements.  Floating point is FP64 throughout.

Modules
  cfe1d     1D convolution-FE space (App. B radial-basis patches, App. C shape
            functions, Sec. 3.3 eq. KxxMxx matrices)
  hashinit  counter-based mode initialisation (splitmix64)
  scheme    problem parameters and the stabilized semi-implicit scheme
            (Sec. 2.5 eq. AC-discrete-semi-stable-K)
  ctd       greedy enrichment + alternating fixed point (Sec. 3.3, App. D)
  fullgrid  full tensor-product CFE solve of the same scheme (tiny grids)
  energy    discrete energy (Sec. 2.1) on the tensor Gauss grid and separated
"""
