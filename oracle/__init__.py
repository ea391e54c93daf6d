"""Plain FP64 CPU oracle for the local multiple traces formulation (MTF).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The product library (``paper_2502_10907_amd``) never routes through
it, and the two share no code: the only common module is ``mtf_inputs``,
which builds seeded meshes and parameters and holds none of the method's
arithmetic.

Everything here is written for a reader checking it against the paper
(Escapil-Inchauspe & Jerez-Hanckes, "Local Multiple Traces Formulation for
Heterogeneous Electromagnetic Scattering: Implementation and
Preconditioning"):

* ``skeleton``   -- Algorithm 1 (normal swaps per subdomain) and the RWG_i
                    spaces of eq. (rwg_multitrace), Section 4.2.
* ``quadrature`` -- the degree-4 triangle rule used on separated pairs and
                    the Sauter--Schwab relative-coordinate rules used on
                    touching pairs (Sauter & Schwab 2011, Section 5.2).
* ``operators``  -- Galerkin blocks of the MFIO K and EFIO T of eq.
                    (boundary_operators), the twisted Gram / transmission
                    blocks of eq. (trick_transmission), the plane-wave
                    right-hand side and the far field.
* ``system``     -- the Galerkin matrix of Problem 2 (Section 3.2), dense
                    LU and plain GMRES.
* ``mie``        -- Mie series of a dielectric sphere (Bohren & Huffman
                    1983, Chapter 4), an external check.

Textbook closed forms that pin the oracle live with the tests
(``tests/_closed_forms.py``), not here.

Where the paper is silent or inconsistent, the reading taken is stated at
the function that takes it.
"""
