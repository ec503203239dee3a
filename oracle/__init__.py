"""CPU FP64 oracle of the qHP TD-CFIE marching-on-in-time method.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, independent
restatement of the method of Le, Cordel, Andriulli and Cools, "A stabilized
time-domain combined field integral equation using the quasi-Helmholtz
projectors" (arXiv 2312.06367), written from the paper's equations.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run it.  The product library never links, imports
or calls anything here, and this package never imports the product.

Parity unpinned (see each module header): the coupling value eta_c, the
quadrature specification and the modulated-pulse definition are readings the
paper leaves open; they are fixed identically on both sides but nothing in the
paper pins their values.
"""
