"""MI355X-native RI qsGW iteration (libqsgw) and its Python binding.

The compiled library lives next to this file (libqsgw.so, built by
``paper_2210_17093_amd.build``); ``paper_2210_17093_amd.qsgw`` binds it.
Importing the binding without the library raises ImportError: there is no
CPU fallback.
"""
__all__ = ["build", "qsgw"]
