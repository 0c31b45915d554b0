"""Exact and prefix-stratified expected values over the Bernoulli paths of a
recombinant binomial tree, on AMD Instinct MI355X (gfx950).

The compute path is the C-ABI library ``libbt.so`` (hand-written HIP);
``paper_1701_03512_amd.bt`` is its ctypes binding.  Importing the package does
not load the library; the first call into ``bt`` does, and raises if it has not
been built.
"""
