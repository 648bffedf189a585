"""CPU oracle for the throughput-distortion GEMM of Anastasia & Andreopoulos,
"Throughput-Distortion Computation of Generic Matrix Multiplication".

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke check of
the entry module and the CPU-baseline leg of the benchmark may import it. The
GPU library never imports, links or calls anything here, and nothing here
imports the GPU library: the two share no code, tables or constants.

It is a plain, slow, obviously-correct numpy implementation of every step of
the method, each function citing the passage of the paper it follows:

* ``exactsum``     exactly rounded sums (used for statistics and control sums)
* ``blocks``       inner-kernel blocking and per-block statistics (Sec. 2, Sec. 3, Sec. 5.B)
* ``packing``      companding (eq. 3), both packing forms (eqs. 6, 7, 11), the
                   packed products (eqs. 8, 12), unpacking (eqs. 9, 10, 13, 14),
                   reverse companding (eq. 5), Prop. 1 (eqs. 15-17)
* ``noise``        quantization / combined noise model (Prop. 2, eqs. 19-21),
                   minimum-error companders (Prop. 4, eq. 26), general
                   companders (Prop. 3, eqs. 22-25)
* ``control``      per-pair option records (Sec. 5.B) and top-down pruning (Sec. 6)
* ``calibration``  representation-noise measurement s(R,W), m(R,W) (Sec. 4.B, eq. 18)
* ``pipeline``     the whole GEMM: stats -> plan -> compand -> pack -> product
                   -> unpack -> de-compand -> l-sum, keeping every intermediate
* ``precision``    the INT8 / FP8 block-scaled form on the same integers (Remark 1)

Readings of passages that are silent, ambiguous or garbled are listed in the
repository's design notes; each function states the reading it takes.
"""
