"""MI355X-native fV-SRN hot path: fused ray-march, point evaluation, forward-mode
density gradients and training kernels for gfx950, behind a C ABI
(``include/fvsrn.h``). The Python layer only marshals arguments."""
