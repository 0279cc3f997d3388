"""FP64 CPU oracle for the batched likelihoods and the nested sampler.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it; the library in
``paper_2509_13307_amd`` never does, and shares no code with it.

Everything is float64 NumPy/SciPy (complex128 where the complex-step gradient
needs it), written from the paper's definitions:

* ``emulator``  : the neural emulator (Sec. 2.2-2.4; CosmoPower-style MLP).
* ``cmb``       : Gaussian CMB-style likelihoods (Sec. 2.3).
* ``shear``     : tomographic cosmic-shear likelihood, Eqs. (A1)-(A4), App. A.
* ``likelihood``: prior transform (Table 1) and the per-model dispatch.
* ``philox``    : the counter-based random number generator both sides use.
* ``nested``    : nested slice sampling with k-deletion and the evidence
                  accumulator (Eq. 1, Sec. 2.1-2.2).
* ``gradient``  : complex-step gradient of the log-likelihood.

Parity status of each function is stated in its docstring; a function whose
result no independent check fixes says "parity unpinned".
"""
