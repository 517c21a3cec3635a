"""FP64 CPU oracle for the Maxwell-Stefan MRT lattice Boltzmann sweep.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written reference
that the HIP path is checked against.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import it;
the product package never does, and nothing here imports the product package.

Contents (each function cites the passage of Chai, Guo, Wang & Shi,
"Maxwell-Stefan theory based lattice Boltzmann model for diffusion in
multicomponent mixtures", that it follows):

* ``lattice``  - velocity sets, weights, opposite directions, the moment
                 matrices M0 (Sec. 3.1, Eqs. (3-5), (3-7), (3-10), (3-14)).
* ``ms``       - the continuum Maxwell-Stefan algebra: matrix B, the
                 generalised Fick matrix, and the map from it to the
                 relaxation matrices (Sec. 2, Eqs. (2-10)-(2-12); Sec. 3,
                 Eqs. (3-16), (3-26)).
* ``lbm``      - initialisation, moment-space collision, propagation with the
                 boundary rules of Sec. 4, observables (Eqs. (3-13), (3-15),
                 (3-27)) and conservation diagnostics, vectorised with numpy.
* ``naive``    - a second, scalar-loop implementation of the same step for
                 brute-force cross-checks on tiny grids.
* ``twin``     - a torch-CPU FP64 twin of the step whose autograd gradients
                 serve as the reference for the hand-written adjoint.

Readings of passages the paper leaves open (lattices other than D2Q5, the
sound speed on D3Q7, the value of lambda_0, node placement, ...) are listed in
the design notes at the repository root.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, analytic solutions, exact symmetries or numbers printed
in the paper; none is "parity unpinned".
"""
