"""MI355X-native throughput-distortion GEMM (Anastasia & Andreopoulos).

The HIP library libtdgemm.so (built from csrc/ by build.py) implements every
step on the GPU; ``tdgemm`` is its Python binding (same entry-point names as
include/tdgemm.h) and ``autograd`` a straight-through linear layer on top of
it. Importing the binding fails if the library has not been built.
"""
