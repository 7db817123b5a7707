"""Build-time generators for the HIP kernels (tables, renaming maps, S-box
gate networks).  They run on the host when the library is built and write
C++ headers under csrc/generated; nothing here runs at encryption time."""
