"""Plain FP64 CPU oracle for randomized tensor-ring decomposition (rTR-ALS / rTR-SVD).

Yuan, Li, Cao, Zhao, "Randomized Tensor Ring Decomposition and Its Application to
Large-scale Data Reconstruction" (arXiv:1901.01652).

This package is TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the GPU library
(it imports nothing from ``paper_1901_01652_amd``) and the GPU library never imports it.

Modules
-------
philox   counter-based Gaussian generator (Philox4x32-10 + Box-Muller), written from the
         published definitions; the Gaussian test matrices of Alg. 1 step 4 come from it.
tensor   definitions of Sec. 2: unfoldings, mode-n product, the TR format Psi (Eq. 1),
         the subchain tensor and the TR unfolding identity (Eq. 2).
rtr      Alg. 1 step by step: sketch, economy QR, power iterations, compression (Eq. 3),
         TR-ALS, TR-SVD, back-projection, RSE.
mlp      FP64 forward/backward of the warm-start network and its TR-reconstruction loss.
sparse   steps 4-7 for a tensor given by its nonzeros (densified, or looped over the entries).

Every function states the passage it follows.  Parity status of each function is listed in
its docstring; functions without an independent pin say "parity unpinned".
"""

