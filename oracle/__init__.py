"""CPU FP64 oracle of mixed-precision block-Jacobi PCG (arXiv 2407.15973).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it. It shares no code, header, table
or helper with the HIP library; its only common dependency is the seeded
input generator module, which holds none of the method's arithmetic.

Everything is plain NumPy in float64 except the storage rounding the method
itself prescribes (reduced-precision block inverses, the FP32 copy of the
residual fed to them), which is emulated exactly. Each function cites the
passage of the paper it follows.

Modules
-------
precision  correctly rounded FP64 -> FP32/BF16/FP16 storage, per-block scale
blocks     diagonal-block extraction, textbook Cholesky inverse, block
           features, per-block precision rule, emulated storage, z = M^-1 r
pcg        preconditioned CG with fMP / aMP(hl) / aMP(lh), the paper's
           polynomial BJAC(k, t) with inner Jacobi sweeps
mlp        16-64-64-3 ReLU MLP, softmax cross-entropy, backward, Adam
labels     per-block precision labels from the method's own runs (a ladder
           of global tolerances, the largest whose delay stays within 5 %)
"""
