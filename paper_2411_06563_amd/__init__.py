"""MI355X (gfx950) implementation of the hot path of the higher-order super-compact
(HOSC) scheme for 3D natural convection of power-law fluids (arXiv 2411.06563).

The compute path is the HIP library ``libhosc.so`` behind the C ABI of
``include/hosc.h``; ``paper_2411_06563_amd.hosc`` is its Python binding."""
