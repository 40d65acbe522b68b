"""Indexed similar-DNA-sequence search (Genoogle, arXiv 1507.02987) on AMD MI355X."""
