"""Levelized static timing analysis on AMD MI355X: Python binding of the libsta C ABI."""
from .sta import (Forward, Graph, SmoothedSlack, StaError, load_library, smoothed_tns, smoothed_wns,
                  STA_CANONICAL_IO, STA_GRAD, STA_GRAD_WNS, STA_RAT, STA_SMOOTH, EXPORTED)

__all__ = ["Forward", "Graph", "SmoothedSlack", "StaError", "load_library", "smoothed_tns", "smoothed_wns",
           "STA_CANONICAL_IO", "STA_GRAD", "STA_GRAD_WNS", "STA_RAT", "STA_SMOOTH", "EXPORTED"]
