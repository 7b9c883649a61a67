"""Levelized static timing analysis on AMD MI355X: Python binding of the libsta C ABI."""
from .place import TimingDescent
from .sta import (Forward, Graph, Server, SmoothedSlack, StaError, load_library, smoothed_tns, smoothed_wns,
                  STA_CANONICAL_IO, STA_GRAD, STA_GRAD_WNS, STA_GRAPH, STA_RAT, STA_SMOOTH, EXPORTED)

__all__ = ["TimingDescent", "Forward", "Graph", "Server", "SmoothedSlack", "StaError", "load_library", "smoothed_tns",
           "smoothed_wns", "STA_CANONICAL_IO", "STA_GRAD", "STA_GRAD_WNS", "STA_GRAPH", "STA_RAT", "STA_SMOOTH",
           "EXPORTED"]
