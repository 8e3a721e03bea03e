"""MI355X-native strength-SPH hot path (arXiv 2603.19764): gfx950 HIP
kernels behind the C-ABI of include/sph.h, with a thin Python binding."""
