"""MI355X-native improved W-stacking (Ye, Gull, Tan & Nikolic 2021): gridding and
degridding behind the C-ABI library libwsgrid.so (include/wsgrid.h).

``paper_2101_11172_amd.wsgrid`` is the binding; ``paper_2101_11172_amd.inputs``
draws the synthetic workloads.  Importing the package loads nothing native; the
binding loads the library on first use and raises if it is missing.
"""
