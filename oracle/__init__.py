"""Plain FP64 CPU oracle for block-level domain decomposition with WaveHoltz
subdomain solves (Rotem, "Efficient Domain Decomposition for the Helmholtz
Equation on GPUs").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path: the only module both
sides read is ``workloads`` (seeded input generators, no method arithmetic).

Contents (each function cites the passage of the paper it follows):

* ``gll``        GLL nodes, weights and the 1D differentiation matrix (Sec. IV).
* ``sem``        Spectral-element assembly of A, M, H and b on a rectangle
                 (Sec. IV, eqs. (3)-(4)) and the global sparse LU solve.
* ``brute``      Dense brute-force element integrals from explicit Lagrange
                 polynomials (an independent check of ``sem``).
* ``dd``         Non-overlapping partition, subdomain systems, the interface
                 exchange (eq. (2)), the exact-solve DD sweep and the outer
                 iteration (fixed point and restarted GMRES, Sec. III).
* ``waveholtz``  The WaveHoltz fixed-point iteration (Sec. V, eqs. (6)-(7),
                 modified leapfrog) and the time-step rule.
* ``sem3``, ``dd3``  The same discretisation and decomposition on a box with
                 hexahedral elements (the 3D workload of Sec. VII-B).

Readings taken where the paper is silent or inconsistent are stated in the
docstrings where they are used (sign of the filter term, the 2/N_t factor,
the sign of the interface update, the time-step rule).

Parity status: every function here is pinned by a ``-m "not gpu"`` test
except the tan^2 constant of the filter, which the fixed point does not
depend on ("parity unpinned" beyond iterate agreement with the GPU path; see
``waveholtz.filter_tables``).
"""
