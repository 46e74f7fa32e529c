"""MI355X (gfx950) implementation of one EMC iteration (arXiv:1409.4256) behind a C ABI.

`emc` is the thin ctypes binding of libemc.so (argument marshalling only);
`build` compiles the HIP sources.
"""
