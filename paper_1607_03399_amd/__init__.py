"""MI355X-native reduced-storage nodal DG for acoustics on vertically mapped wedges.

The compute path is the HIP library ``libwdg.so`` (C ABI in ``include/wdg.h``);
``paper_1607_03399_amd.wdg`` is its thin ctypes binding.  Importing the
package loads nothing; the binding loads the library on first use and
raises if it has not been built.
"""
