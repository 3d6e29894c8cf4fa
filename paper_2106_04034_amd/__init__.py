"""MI355X-native (gfx950, HIP) hot path of Geometric Semantic Genetic
Programming (GSGP-CUDA, arXiv 2106.04034).

``paper_2106_04034_amd.gsgp`` is the binding of libgsgp.so (include/gsgp.h);
``paper_2106_04034_amd.synth`` draws seeded synthetic workloads;
``paper_2106_04034_amd.build`` compiles the library with hipcc;
``paper_2106_04034_amd.cases`` reads and writes the paper's text formats, and
``python -m paper_2106_04034_amd`` runs GSGP on them from the command line.
Importing the package loads nothing; the library is loaded on first use.
"""
__all__ = ["gsgp", "synth", "build", "cases"]
