"""MI355X-native exact-exchange library: batched Kronecker-product Poisson
solves for Vx.psi (arXiv 2501.16572), hand-written HIP kernels for gfx950
behind a C ABI (``libkronx.so``).  ``kronx`` is the thin Python binding."""
