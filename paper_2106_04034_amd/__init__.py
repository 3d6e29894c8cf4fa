"""MI355X-native (gfx950, HIP) hot path of Geometric Semantic Genetic
Programming (GSGP-CUDA, arXiv 2106.04034).

``paper_2106_04034_amd.gsgp`` is the binding of libgsgp.so (include/gsgp.h);
``paper_2106_04034_amd.synth`` draws seeded synthetic workloads;
``paper_2106_04034_amd.build`` compiles the library with hipcc.
Importing the package loads nothing; the library is loaded on first use.
"""
__all__ = ["gsgp", "synth", "build"]
