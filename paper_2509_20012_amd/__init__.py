"""MI355X-native hot path of superiorized feasibility-seeking dose/LETd plan
optimization (arXiv 2509.20012): CSR/CSC influence-matrix kernels in HIP for gfx950
behind a C ABI, with a thin Python binding."""
