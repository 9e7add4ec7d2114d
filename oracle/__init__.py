"""CPU FP64 oracle for MPS Pauli-pair feature extraction -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke entry point and the benchmark's CPU baseline may import this
package.  The device library never calls it and shares no code with it.

Modules (each function cites the passage of the paper it follows):

* ``gates``        -- one- and two-qubit gate matrices and the Pauli basis (§II-A, §II-C).
* ``statevector``  -- plain statevector simulation, n <= 20 (the baseline backend of §I/§III),
                      and two-site reduced density matrices.
* ``bruteforce``   -- full 2^n x 2^n unitary from Kronecker products, n <= 10 (independent
                      second statevector path used only to pin ``statevector``).
* ``mps``          -- matrix product state simulation (Eq. (3)): local one-qubit updates,
                      two-site update + SVD truncation to at most chi (§II-B), environment
                      sweeps and transfer-matrix pair density matrices.
* ``closed_form``  -- exact closed forms at L = 0 (product state) and L = 1 (Clifford
                      conjugation through the CNOT ladder), any n.
* ``readout``      -- Pauli-basis coefficients of the adaptive observables (Eq. (4)),
                      features by linearity (Eq. (5)) and the linear reconstruction (Eq. (6)).
* ``features``     -- front door: exact or truncated Pauli-pair features for a batch.

Parity unpinned: truncated results whose kept/discarded singular values are (nearly)
degenerate are only bound-checked (the truncation is not unique there).
"""
