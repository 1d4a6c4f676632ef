"""CPU oracle for the EPRL vertex tensor in the booster decomposition.

This package is test infrastructure. It is a plain, slow, deliberately unoptimised
restatement of what the paper (Gozzini, "A high-performance code for EPRL spin foam
amplitudes", arXiv:2107.13952) defines, used only to check the HIP library:

* ``wigner``   - exact Racah-formula 6j symbols (big integers / Fractions), Sec. 2 and the
                 6j symbols entering eq. (15j).
* ``ranges``   - intertwiner ranges, virtual-spin shells, packed booster layout (Sec. 2,
                 eq. (vertex-ampl); Sec. 3.1 "Tensor contractions", framed algorithm,
                 steps 1-3).
* ``fifteenj`` - the {15j} symbol of the first kind as a sum over x of five 6j
                 symbols, eq. (15j).
* ``vertex``   - the vertex tensor A(i1..i5), eq. (vertex-ampl), computed shell by shell
                 as in the framed algorithm of Sec. 3.1 (steps 5-7).
* ``contract`` - the contraction of A with five boundary vectors (Sec. 3.2, the
                 ``contract`` call) and its derivatives.
* ``boosters`` - the booster functions of eq. (booster) by FP64 quadrature (Sec. 3.1,
                 "Booster coefficients"): the input the library takes, produced for the
                 parity cases and the benchmark.

Only ``tests/``, the smoke entry point and the CPU-baseline leg of the benchmark may import
it. The GPU product path never does, and this package never imports the GPU path.
"""
