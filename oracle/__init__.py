"""CPU oracle for the QUAPI reduced-density-matrix propagation (FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links
or executes anything in this package: only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP path (no kernels, headers, helpers, tables or constants).

What it computes (all in float64 / complex128, hbar = k_B = 1):

* ``bath``   the lineshape G(t) = double time integral of the bath response
             alpha(t) (Sec. II, bath-response equation), in closed form for
             the Ohmic spectral density and by adaptive quadrature for a
             tabulated J(omega); alpha(t) itself by quadrature.
* ``eta``    the eta coefficients of the discretized influence functional
             (Sec. II, the eta_kk' ... eta_Nk definitions) from G, both by
             class (second differences on the half-step grid) and for an
             arbitrary pair of path points from their time intervals.
* ``system`` the bare propagator exp(-i H dt) and the Liouville-space
             propagator K (Sec. II, the exact path-sum equation), and the
             influence factors F_eta.
* ``brute``  the discretized, memory-truncated path sum enumerated over all
             paths (tiny cases).
* ``tensor`` the same sum by the tensor-propagator recursion (plain C, with
             OpenMP over output entries), for the workload sizes.
* ``entry``  one output entry of one propagation step, by definition.
* ``run``    end-to-end: inputs -> rho(t_k), k = 0..n.

Parity pins live in ``tests/test_oracle_*.py``.  No function here is
"parity unpinned"; every one is checked against a closed form, a limit, an
invariant, brute force, or a value printed in the paper.
"""
from . import bath, eta, system, brute, tensor, entry, run  # noqa: F401
from .run import oracle_run, OracleInputs  # noqa: F401
