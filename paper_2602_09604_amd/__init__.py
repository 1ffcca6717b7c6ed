"""MI355X state-vector gate application: C-ABI library ``libsv.so`` plus a thin
ctypes binding (``paper_2602_09604_amd.sv``).  Importing this package does not
load the library; the binding loads it on first use and raises if it is
missing."""
__version__ = "0.1.0"
