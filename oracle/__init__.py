"""Plain FP64 CPU oracle of the energy-based FEM hot path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product path (``paper_2602_12365_amd``) never imports it, and
this package imports nothing from the product path; inputs reach both sides as
plain numpy arrays.

* ``oracle.fem``    element operators (energy, residual, tangent action,
                    Jacobi diagonal, material and coordinate adjoints) for the
                    neo-Hookean and linear-elastic densities in plain C
                    (``efem_oracle.c``), Dirichlet condensation, Newton-CG.
* ``oracle.mlp``    forward and backward of the per-node MLP in FP64 numpy.
* ``oracle.precond`` node features of the learned preconditioner.
* ``oracle.transport`` the non-variational transport operator (virtual work,
                    Sec. 3.1, Eqs. 4-6; example of Sec. 6.5): residual, element matrices, direct reduced solve.

Every function cites the passage of the paper it follows.  Functions with no
independent pin say "parity unpinned" in their docstring.
"""
