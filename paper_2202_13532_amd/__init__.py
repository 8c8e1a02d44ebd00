"""MI355X (gfx950) tensor-product nodal DG Vlasov-Poisson hot path.

The compute path is the HIP library ``libdg.so`` (C ABI in include/dg.h);
``paper_2202_13532_amd.dg`` is its thin ctypes binding.  ``inputs`` and
``workloads`` describe synthetic problems.  Importing the package does not load
the library; the first call into ``dg`` does, and fails loudly if it is absent.
"""
