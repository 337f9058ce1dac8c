"""Learned tile / theta-band proposal: the CNN (ProposalNet), its training
from plain-pipeline labels, and the evaluation of the pruned vote."""
