"""CPU oracle for FNO-EOM-CCSDT (test infrastructure, FP64, slow by design).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is an independent, plain
implementation of what the GPU library computes and shares no code with it:

* ``det``  -- determinant-space brute force of the definitions (eqs 1-7) and FCI;
* ``wick`` -- Wick's-theorem expansion of eq (5) and of the EOM sigma vectors;
* ``cc``   -- CCSDT residuals/energy, Jacobi+DIIS, EOM sigma, Davidson, dense EOM;
* ``fno``  -- MP2 amplitudes, virtual density and FNO truncation (eqs 8-10);
* ``mlp``  -- the learned-guess network (forward, backpropagation) and its training data;
* ``xfno`` -- XFNO: FNO energies at several thresholds and their linear extrapolation.
"""
