"""FP64 CPU oracle of the particle-mesh (PM) kick-drift-kick method.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the entry
module and the CPU-baseline leg of the benchmark may import this package.  The
product path (the HIP library and its Python binding) never calls it and
shares no code with it.

The oracle is deliberately plain and slow: NumPy/SciPy in float64, library
FFTs (``scipy.fft``) as single steps, no blocking, fusion or reordering beyond
what the method states.  Each function cites the passage of the paper
(Modi, Lanusse & Seljak, "FlowPM: Distributed TensorFlow implementation of the
FastPM cosmological N-body solver", arXiv:2010.11847) that it follows; where
the paper defers to FastPM (Feng et al. 2016) the formula is derived from the
equations of motion and linear theory and marked *derived*.

Modules
-------
cosmology : background expansion, growth factors, FastPM kick/drift factors,
            linear power spectra and sigma8 normalisation.
rng       : counter-based white noise (SplitMix64 finaliser + Box-Muller).
lpt       : Gaussian linear field and 1LPT/2LPT initial conditions (Gen-IC).
pm        : CIC paint/readout, FD Green's function force, KDK integration.
power     : binned power spectrum, transfer function and cross-correlation.
adjoint   : reverse-mode derivative of the whole run (vector-Jacobian products).

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against closed forms, brute force, invariants or library routines, except
where a function header says "parity unpinned".
"""
