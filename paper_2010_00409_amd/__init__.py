"""MI355X implementation of tight focusing by mapping to periodic space
(arXiv:2010.00409).  The compute lives in libtfocus.so (HIP, gfx950); the
``tfocus`` module is its ctypes binding."""
__version__ = "0.1"
