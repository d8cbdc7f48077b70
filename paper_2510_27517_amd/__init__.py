"""MI355X (gfx950) preconditioned conjugate gradient with a factorized sparse
approximate inverse, M^-1 = G G^T + eps I.

Modules:
  pcg     - binding of the C ABI (include/pcg.h) implemented by libpcg.so
  inputs  - seeded synthetic systems (2D/3D Poisson, RGG Laplacian, elasticity)
  build   - in-tree compilation of libpcg.so for gfx950
"""
