"""FP64 CPU oracle for the DiFVM hot path (test infrastructure; see oracle.cpp's header)."""
