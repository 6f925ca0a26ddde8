"""CPU oracle for the sliced-stem contraction: test infrastructure only.

Plain, slow, FP64 NumPy code that computes what the GPU path must reproduce,
written from the paper's definitions.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import this package; the product
path never calls it and shares no code with it (both read the seeded inputs
of ``workloads/`` as data).

Modules:

* ``gates``       -- gate matrices of paper §2.
* ``statevector`` -- FP64 state-vector simulation of a circuit (paper §2).
* ``network``     -- the circuit as a tensor network; its value by the
                     literal Feynman-path sum (§A.1, the value T_H) and by
                     pairwise contraction in any order (§3, Schroedinger
                     method; order independence §A.1).
* ``stemnet``     -- value of a stem network: an initial stem that absorbs
                     branch tensors one after another, for one assignment of
                     the sliced and projected labels (§A.1 slicing, §A.2
                     stems and branches, §A.3 branch pre-computation).
* ``stats``       -- XEB (§2), Porter-Thomas check (§3 and §A.4), relative
                     L2 error.
* ``cost``        -- time complexity and contraction width of a contraction
                     scheme (§A.1).
* ``dense``       -- plain definitions of the two kernels of one stem step:
                     a bit permutation of a tensor and a complex matrix
                     product.
* ``mlp``         -- FP64 reference of the runtime-model network (forward,
                     backward, Adam update).

Parity status of every function is stated in its module docstring.
"""
